// Launch-shape autotuner: times every supported (block, draws per lane,
// unroll) shape of a model class on a probe workload and keeps the fastest.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pps.h"
#include "pps_launch.hpp"
#include "pps_runtime.hpp"

using namespace pps;

namespace {

std::vector<SimShape> candidate_shapes(int cls)
{
    std::vector<SimShape> out;
    for (int block : {64, 128, 256, 512, 1024})
        for (int dpl : {1, 2})
            for (int unroll : {1, 2}) {
                SimShape sh;
                sh.block = block;
                sh.dpl = dpl;
                sh.unroll = unroll;
                if (sim_shape_supported(cls, sh))
                    out.push_back(sh);
            }
    return out;
}

int steps_bucket(int steps)
{
    int b = 1;
    while (b < steps && b < (1 << 30))
        b <<= 1;
    return b;
}

// Draw counts rounded up to a power of two: the best shape of a class moves
// with the job size (tile counts per workgroup and the grid's last round).
uint64_t draws_bucket(uint64_t n)
{
    uint64_t b = 1;
    while (b < n && b < (uint64_t(1) << 62))
        b <<= 1;
    return b;
}

std::string arch_name(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Cache file lines: "<arch> <class> <steps bucket> <draws bucket> <block>
// <dpl> <unroll> <ms>"; lines of any other form are skipped.
bool cache_lookup(const char *path, const std::string &arch, int cls, int bucket,
                  unsigned long long dbucket, SimShape *sh)
{
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char line[256], a[64];
    int c, b, block, dpl, unroll;
    unsigned long long db;
    double ms;
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%63s %d %d %llu %d %d %d %lf", a, &c, &b, &db, &block, &dpl, &unroll,
                        &ms) != 8)
            continue;
        if (arch == a && c == cls && b == bucket && db == dbucket) {
            sh->block = block;
            sh->dpl = dpl;
            sh->unroll = unroll;
            found = sim_shape_supported(cls, *sh);  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_append(const char *path, const std::string &arch, int cls, int bucket,
                  unsigned long long dbucket, const SimShape &sh, double ms)
{
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f, "%s %d %d %llu %d %d %d %.6f\n", arch.c_str(), cls, bucket, dbucket, sh.block,
                 sh.dpl, sh.unroll, ms);
    std::fclose(f);
}

}  // namespace

extern "C" int pps_autotune(const pps_model *model, uint64_t n_draws, int use_cache,
                            pps_tune_report *report, void *stream)
{
    clear_error();
    int ns = 0, rc;
    if ((rc = validate_model(model, &ns)) != PPS_OK)
        return rc;
    if (n_draws == 0)
        return fail(PPS_EINVAL, "pps_autotune: n_draws must be >= 1");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    const int cls = model_class(model);
    const int steps = model->model == PPS_NORMAL_MEAN ? model->n_obs : model->steps;
    const int bucket = steps_bucket(steps);
    const unsigned long long dbucket = draws_bucket(n_draws);
    const std::string arch = arch_name(c->device);
    const char *cache = std::getenv("PPS_TUNE_CACHE");
    if (report) {
        std::memset(report, 0, sizeof *report);
        report->model_class = cls;
        report->best = -1;
    }
    SimShape cached;
    if (use_cache && cache && cache_lookup(cache, arch, cls, bucket, dbucket, &cached)) {
        c->engine->set_shape(cls, cached);
        if (report) {
            report->n_entries = 1;
            report->entries[0] = {cached.block, cached.dpl, cached.unroll, -1.0};
            report->best = 0;
            report->from_cache = 1;
        }
        return PPS_OK;
    }

    if (c->counts.ensure(PPS_GARCH_NSUMM * sizeof(unsigned long long)) != hipSuccess)
        return fail(PPS_ENOMEM, "pps_autotune: tally buffer");
    pps_sampling s;
    s.n_draws = n_draws;
    s.first_draw = 0;
    s.seed = 0x5eedull;
    const std::vector<SimShape> shapes = candidate_shapes(cls);
    const SimShape keep = c->engine->shape(cls);
    double best_ms = INFINITY;
    int best = -1;
    for (size_t i = 0; i < shapes.size(); ++i) {
        c->engine->set_shape(cls, shapes[i]);
        double ms_best = INFINITY;
        for (int rep = 0; rep < 3; ++rep) {  // first run warms up (graph capture, code load)
            EpochPlan plan;
            JobDev J;
            fill_job(J, model, &s, ns, cls == CLASS_GARCH ? JOB_TALLY_SUMM : JOB_TALLY_STAT);
            J.counts = c->counts.as<unsigned long long>();
            J.n_counts = cls == CLASS_GARCH ? PPS_GARCH_NSUMM : 1;
            J.row_flags = ROW_ZERO_COUNTS;
            J.tile_offset = 0;
            J.n_tiles = c->engine->tiles_for(cls, n_draws);
            plan.rows[cls].push_back(J);
            if ((rc = c->engine->launch(0, plan, static_cast<hipStream_t>(stream))) != PPS_OK ||
                (rc = c->engine->wait(0)) != PPS_OK) {
                c->engine->set_shape(cls, keep);
                return rc;
            }
            if (rep > 0 && c->engine->sim_ms(0) > 0.0f)
                ms_best = std::fmin(ms_best, c->engine->sim_ms(0));
        }
        if (report && i < 16) {
            report->entries[i] = {shapes[i].block, shapes[i].dpl, shapes[i].unroll, ms_best};
            report->n_entries = static_cast<int32_t>(i + 1);
        }
        if (ms_best < best_ms) {
            best_ms = ms_best;
            best = static_cast<int>(i);
        }
    }
    if (best < 0) {
        c->engine->set_shape(cls, keep);
        return fail(PPS_EDEVICE, "pps_autotune: no shape could be timed");
    }
    c->engine->set_shape(cls, shapes[best]);
    if (report)
        report->best = best;
    if (cache)
        cache_append(cache, arch, cls, bucket, dbucket, shapes[best], best_ms);
    return PPS_OK;
}
