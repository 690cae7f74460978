// extern "C" entry points of libpps (declared in include/pps.h).  Every
// synchronous call builds one epoch plan and runs it through the calling
// device's epoch engine (one captured graph), then reads the staged results.
#include <cmath>
#include <cstring>
#include <vector>

#include "pps.h"
#include "pps_launch.hpp"
#include "pps_runtime.hpp"

using namespace pps;

#define PPS_TRY_HIP(expr, what)                                                                \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail_hip(e_, what);                                                         \
    } while (0)

#define PPS_TRY(expr)                                                                          \
    do {                                                                                       \
        int rc_ = (expr);                                                                      \
        if (rc_ != PPS_OK)                                                                     \
            return rc_;                                                                        \
    } while (0)

static hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

static void whole_job(const EpochEngine &eng, int cls, JobDev &row)
{
    row.tile_offset = 0;
    row.n_tiles = eng.tiles_for(cls, row.n_draws);
}

// Runs one plan to completion on `stream` (context lock held by the caller).
static int run_sync(Context &c, EpochPlan &plan, hipStream_t stream)
{
    PPS_TRY(c.engine->launch(0, plan, stream));
    PPS_TRY(c.engine->wait(0));
    if (g_timing)
        c.last_kernel_ms = c.engine->sim_ms(0);
    return PPS_OK;
}

namespace pps {

int abc_check(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
              int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
              float *acc_theta, float *acc_dist, const pps_abc_stats *stats, int *n_summ)
{
    PPS_TRY(validate_model(model, n_summ));
    PPS_TRY(validate_sampling(sampling));
    if (!stats)
        return fail(PPS_EINVAL, "abc_sample: stats is required");
    PPS_TRY(validate_abc(model, y_obs, *n_summ, sampling, eps_mode, eps_or_frac));
    if (capacity > 0 && (!acc_idx || !acc_theta || !acc_dist))
        return fail(PPS_EINVAL, "abc_sample: output buffers required when capacity > 0");
    return PPS_OK;
}

int abc_run(Context &c, const pps_model *model, int n_summ, const double *y_obs,
            const pps_sampling *sampling, int eps_mode, double eps_or_frac, uint64_t capacity,
            uint64_t *acc_idx, float *acc_theta, float *acc_dist, pps_abc_stats *stats,
            void *scratch, EpochPlan &plan, bool build, hipStream_t stream)
{
    const AbcScratch scr = abc_scratch_at(scratch, sampling->n_draws);
    plan.clear();
    JobDev J;
    fill_job(J, model, sampling, n_summ, JOB_WRITE_DIST);
    for (int k = 0; k < n_summ; ++k)
        J.y_obs[k] = static_cast<float>(y_obs[k]);
    J.dist = scr.dist;
    const int cls = model_class(model);
    whole_job(*c.engine, cls, J);
    plan.rows[cls].push_back(J);
    FinJob F;
    fill_fin(F, J, eps_mode, eps_or_frac, capacity, acc_idx, acc_theta, acc_dist, scr);
    plan.fins.push_back(F);
    PPS_TRY(c.engine->launch(0, plan, stream, build));
    PPS_TRY(c.engine->wait(0));
    if (g_timing) {
        c.last_kernel_ms = c.engine->sim_ms(0);
        c.last_finalize_ms = c.engine->fin_ms(0);
    }

    const FinResult &R = c.engine->out_fin(0)[0];
    stats->n_accepted = R.n_accepted;
    stats->eps_used = R.eps_used;
    for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
        stats->mean[j] = R.mean[j];
        stats->var[j] = R.var[j];
    }
    if (R.n_accepted > capacity)
        return fail(PPS_ETRUNC, "abc_sample: %llu accepted, capacity %llu",
                    static_cast<unsigned long long>(R.n_accepted),
                    static_cast<unsigned long long>(capacity));
    return PPS_OK;
}

}  // namespace pps

extern "C" {

const char *pps_version(void) { return "pps 0.2 (gfx950)"; }

const char *pps_last_error(void) { return last_error(); }

int pps_set_timing(int enable)
{
    g_timing = enable != 0;
    return PPS_OK;
}

double pps_last_finalize_ms(void)
{
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return -1.0;
    std::lock_guard<std::mutex> lk(c->mu);
    return c->last_finalize_ms;
}

double pps_last_kernel_ms(void)
{
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return -1.0;
    std::lock_guard<std::mutex> lk(c->mu);
    return c->last_kernel_ms;
}

int pps_set_block_size(int model_class, int block)
{
    clear_error();
    if (model_class < 0 || model_class >= N_CLASSES)
        return fail(PPS_EINVAL, "unknown model class %d", model_class);
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    SimShape sh = c->engine->shape(model_class);
    sh.block = block;
    if (!sim_shape_supported(model_class, sh))
        return fail(PPS_EINVAL, "block size %d not supported for class %d", block, model_class);
    c->engine->set_shape(model_class, sh);
    return PPS_OK;
}

int pps_get_block_size(int model_class)
{
    clear_error();
    if (model_class < 0 || model_class >= N_CLASSES)
        return fail(PPS_EINVAL, "unknown model class %d", model_class);
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    return c->engine->shape(model_class).block;
}

int pps_set_launch_shape(int model_class, int block, int draws_per_lane, int unroll)
{
    clear_error();
    if (model_class < 0 || model_class >= N_CLASSES)
        return fail(PPS_EINVAL, "unknown model class %d", model_class);
    SimShape sh;
    sh.block = block;
    sh.dpl = draws_per_lane;
    sh.unroll = unroll;
    if (!sim_shape_supported(model_class, sh))
        return fail(PPS_EINVAL, "launch shape (%d, %d, %d) not supported for class %d", block,
                    draws_per_lane, unroll, model_class);
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    c->engine->set_shape(model_class, sh);
    return PPS_OK;
}

int pps_get_launch_shape(int model_class, int *block, int *draws_per_lane, int *unroll)
{
    clear_error();
    if (model_class < 0 || model_class >= N_CLASSES)
        return fail(PPS_EINVAL, "unknown model class %d", model_class);
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    const SimShape &sh = c->engine->shape(model_class);
    if (block)
        *block = sh.block;
    if (draws_per_lane)
        *draws_per_lane = sh.dpl;
    if (unroll)
        *unroll = sh.unroll;
    return PPS_OK;
}

const char *pps_strerror(int status)
{
    switch (status) {
    case PPS_OK: return "ok";
    case PPS_PENDING: return "pending";
    case PPS_EINVAL: return "invalid argument";
    case PPS_ENOMEM: return "out of memory";
    case PPS_EDEVICE: return "device error";
    case PPS_EBUSY: return "busy";
    case PPS_ENOTFOUND: return "not found";
    case PPS_ETRUNC: return "output truncated to capacity";
    default: return "unknown status";
    }
}

int pps_n_summaries(const pps_model *model)
{
    clear_error();
    int ns = 0;
    int rc = validate_model(model, &ns);
    return rc == PPS_OK ? ns : rc;
}

int pps_philox(uint64_t seed, uint64_t first_draw, uint64_t n, uint32_t block, uint32_t purpose,
               uint32_t *out, void *stream)
{
    clear_error();
    if (n == 0 || !out)
        return fail(PPS_EINVAL, "pps_philox: n == 0 or out == NULL");
    PPS_TRY_HIP(launch_philox(seed, first_draw, n, block, purpose, out, as_stream(stream)),
                "pps_philox launch");
    PPS_TRY_HIP(hipStreamSynchronize(as_stream(stream)), "pps_philox");
    return PPS_OK;
}

int pps_normals(uint64_t seed, uint64_t first_draw, uint64_t n, uint32_t m, float *out,
                void *stream)
{
    clear_error();
    if (n == 0 || m == 0 || !out)
        return fail(PPS_EINVAL, "pps_normals: n == 0, m == 0 or out == NULL");
    PPS_TRY_HIP(launch_normals(seed, first_draw, n, m, out, as_stream(stream)),
                "pps_normals launch");
    PPS_TRY_HIP(hipStreamSynchronize(as_stream(stream)), "pps_normals");
    return PPS_OK;
}

int pps_simulate(const pps_model *model, const pps_sampling *sampling, const double *y_obs,
                 float *theta, float *summ, float *stat, float *dist, void *stream)
{
    clear_error();
    int ns = 0, rc;
    PPS_TRY(validate_model(model, &ns));
    PPS_TRY(validate_sampling(sampling));
    if (dist && !y_obs)
        return fail(PPS_EINVAL, "pps_simulate: dist requested without y_obs");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    const int cls = model_class(model);
    EpochPlan plan;
    JobDev J;
    fill_job(J, model, sampling, ns, JOB_DUMP);
    if (y_obs && model->model != PPS_GARCH11)
        for (int k = 0; k < ns; ++k)
            J.y_obs[k] = static_cast<float>(y_obs[k]);
    J.dump_theta = theta;
    J.dump_summ = summ;
    J.dump_stat = model->model == PPS_GARCH11 ? nullptr : stat;
    J.dump_dist = model->model == PPS_GARCH11 ? nullptr : dist;
    whole_job(*c->engine, cls, J);
    plan.rows[cls].push_back(J);
    return run_sync(*c, plan, as_stream(stream));
}

int abc_sample(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
               int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
               float *acc_theta, float *acc_dist, pps_abc_stats *stats, void *stream)
{
    clear_error();
    int ns = 0, rc;
    PPS_TRY(abc_check(model, y_obs, sampling, eps_mode, eps_or_frac, capacity, acc_idx, acc_theta,
                      acc_dist, stats, &ns));
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    PPS_TRY_HIP(c->dist.ensure(abc_scratch_bytes(sampling->n_draws)), "ABC scratch");
    EpochPlan plan;
    return abc_run(*c, model, ns, y_obs, sampling, eps_mode, eps_or_frac, capacity, acc_idx,
                   acc_theta, acc_dist, stats, c->dist.p, plan, true, as_stream(stream));
}

int prior_pred_pvalue(const pps_model *model, int lambda_param, int lambda_family,
                      const double *lambda, int n_lambda, const pps_sampling *sampling,
                      double t_obs, uint64_t *count_ge, double *pvalue, void *stream)
{
    clear_error();
    int ns = 0, rc;
    PPS_TRY(validate_model(model, &ns));
    PPS_TRY(validate_sampling(sampling));
    if (model->model == PPS_GARCH11)
        return fail(PPS_EINVAL, "prior_pred_pvalue: use pps_summary_tally for GARCH");
    if (lambda_param < 0 || lambda_param >= model->n_params)
        return fail(PPS_EINVAL, "lambda_param %d out of range", lambda_param);
    if (lambda_family < PPS_UNIFORM || lambda_family > PPS_POINT)
        return fail(PPS_EINVAL, "unknown lambda_family %d", lambda_family);
    if (!lambda || n_lambda < 1 || n_lambda > 4096)
        return fail(PPS_EINVAL, "n_lambda must be in [1, 4096] with a lambda array");
    if (!count_ge || !pvalue)
        return fail(PPS_EINVAL, "count_ge and pvalue are required");
    if (std::isnan(t_obs))
        return fail(PPS_EINVAL, "t_obs is NaN");
    std::vector<pps_model> mk(n_lambda, *model);
    for (int k = 0; k < n_lambda; ++k) {
        mk[k].prior[lambda_param].family = lambda_family;
        mk[k].prior[lambda_param].b = lambda[k];
        int ns2 = 0;
        if (validate_model(&mk[k], &ns2) != PPS_OK)
            return fail(PPS_EINVAL, "lambda[%d] = %g gives an invalid prior", k, lambda[k]);
    }
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    PPS_TRY_HIP(c->counts.ensure(n_lambda * sizeof(unsigned long long)), "tally buffer");
    // Logistic grids run in groups of GROUP_LPL lambda values sharing each
    // draw's random numbers; the rest (and other models) one row per lambda.
    const int grouped = model->model == PPS_LOGISTIC_SDE ? (n_lambda / GROUP_LPL) * GROUP_LPL : 0;
    EpochPlan plan;
    std::vector<std::pair<int, size_t>> where(n_lambda);  // (class, row index)
    for (int k = 0; k < n_lambda; ++k) {
        const int cls = k < grouped ? CLASS_GROUP : model_class(model);
        JobDev J;
        fill_job(J, &mk[k], sampling, ns, JOB_TALLY_STAT);
        J.t_obs = t_obs;
        J.counts = c->counts.as<unsigned long long>() + k;
        J.n_counts = 1;
        J.row_flags = ROW_ZERO_COUNTS | ROW_COPY_COUNTS;
        J.lambda_param = lambda_param;
        whole_job(*c->engine, cls, J);
        where[k] = {cls, plan.rows[cls].size()};
        plan.rows[cls].push_back(J);
    }
    PPS_TRY(run_sync(*c, plan, as_stream(stream)));
    const unsigned long long *cnt = c->engine->out_counts(0);
    for (int k = 0; k < n_lambda; ++k) {
        const JobDev &R = plan.rows[where[k].first][where[k].second];
        count_ge[k] = cnt[R.out_slot];
        pvalue[k] = static_cast<double>(count_ge[k]) / static_cast<double>(sampling->n_draws);
    }
    return PPS_OK;
}

int pps_summary_tally(const pps_model *model, const pps_sampling *sampling,
                      const double *obs_summ, uint64_t *count_ge, void *stream)
{
    clear_error();
    int ns = 0, rc;
    PPS_TRY(validate_model(model, &ns));
    PPS_TRY(validate_sampling(sampling));
    if (model->model != PPS_GARCH11 && model->model != PPS_TOGGLE_SWITCH && model->model != PPS_TB)
        return fail(PPS_EINVAL, "pps_summary_tally: GARCH, toggle-switch and tuberculosis models only");
    if (!obs_summ || !count_ge)
        return fail(PPS_EINVAL, "obs_summ and count_ge are required");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    PPS_TRY_HIP(c->counts.ensure(ns * sizeof(unsigned long long)), "tally buffer");
    EpochPlan plan;
    JobDev J;
    fill_job(J, model, sampling, ns, JOB_TALLY_SUMM);
    for (int k = 0; k < ns; ++k)
        J.summ_obs[k] = obs_summ[k];
    J.counts = c->counts.as<unsigned long long>();
    J.n_counts = static_cast<uint32_t>(ns);
    J.row_flags = ROW_ZERO_COUNTS | ROW_COPY_COUNTS;
    const int cls = model_class(model);
    whole_job(*c->engine, cls, J);
    plan.rows[cls].push_back(J);
    PPS_TRY(run_sync(*c, plan, as_stream(stream)));
    std::memcpy(count_ge, c->engine->out_counts(0), ns * sizeof(unsigned long long));
    return PPS_OK;
}

int pps_tb_events(const pps_model *model, const pps_sampling *sampling, uint64_t *events,
                  int32_t *status, void *stream)
{
    clear_error();
    int ns = 0, rc;
    PPS_TRY(validate_model(model, &ns));
    PPS_TRY(validate_sampling(sampling));
    if (model->model != PPS_TB)
        return fail(PPS_EINVAL, "pps_tb_events: tuberculosis model only");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    const int cls = model_class(model);
    EpochPlan plan;
    JobDev J;
    fill_job(J, model, sampling, ns, JOB_EVENTS);
    J.dump_events = reinterpret_cast<unsigned long long *>(events);
    J.dump_status = status;
    whole_job(*c->engine, cls, J);
    plan.rows[cls].push_back(J);
    return run_sync(*c, plan, as_stream(stream));
}

}  // extern "C"
