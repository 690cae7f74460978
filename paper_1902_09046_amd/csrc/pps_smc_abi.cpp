// extern "C" entry points of the weak-informativity test (declared in
// include/pps.h): validation, scratch and the launches of pps_smc.hip.
#include <cmath>
#include <cstring>
#include <vector>

#include "pps.h"
#include "pps_runtime.hpp"
#include "pps_smc.hpp"

using namespace pps;

namespace {

int validate_bio(const pps_bioassay *b, BioDesign *out)
{
    if (!b)
        return fail(PPS_EINVAL, "bioassay model is NULL");
    if (b->n_groups < 1 || b->n_groups > PPS_BIO_MAX_GROUPS)
        return fail(PPS_EINVAL, "n_groups %d out of range [1, %d]", b->n_groups, PPS_BIO_MAX_GROUPS);
    std::memset(out, 0, sizeof *out);
    out->n_groups = b->n_groups;
    for (int i = 0; i < b->n_groups; ++i) {
        if (b->n_trials[i] < 0 || b->n_trials[i] > 1000)
            return fail(PPS_EINVAL, "n_trials[%d] = %d out of range [0, 1000]", i, b->n_trials[i]);
        if (!std::isfinite(b->dose[i]))
            return fail(PPS_EINVAL, "dose[%d] is not finite", i);
        out->n_trials[i] = b->n_trials[i];
        out->dose[i] = b->dose[i];
    }
    return PPS_OK;
}

int validate_smc(const pps_smc_config *c, SmcParams *out)
{
    if (!c)
        return fail(PPS_EINVAL, "SMC config is NULL");
    if (c->n_particles < 2 || c->n_particles > PPS_SMC_MAX_PARTICLES)
        return fail(PPS_EINVAL, "n_particles %d out of range [2, %d]", c->n_particles,
                    PPS_SMC_MAX_PARTICLES);
    if (c->max_mcmc < 1 || c->max_mcmc > SMC_BLOCKS_PER_STEP)
        return fail(PPS_EINVAL, "max_mcmc %d out of range [1, %d]", c->max_mcmc, SMC_BLOCKS_PER_STEP);
    if (c->max_steps < 1 || c->max_steps > 4096)
        return fail(PPS_EINVAL, "max_steps %d out of range [1, 4096]", c->max_steps);
    if (c->bisect_iters < 1 || c->bisect_iters > 64)
        return fail(PPS_EINVAL, "bisect_iters %d out of range [1, 64]", c->bisect_iters);
    if (!(c->c > 0.0 && c->c < 1.0))
        return fail(PPS_EINVAL, "c must be in (0, 1)");
    if (!(c->h > 0.0) || !std::isfinite(c->h))
        return fail(PPS_EINVAL, "h must be finite and > 0");
    out->n_particles = c->n_particles;
    out->max_mcmc = c->max_mcmc;
    out->max_steps = c->max_steps;
    out->bisect_iters = c->bisect_iters;
    out->c = c->c;
    out->h = c->h;
    return PPS_OK;
}

int check_lambdas(const double *lam, uint64_t rows)
{
    if (!lam)
        return fail(PPS_EINVAL, "lambda is NULL");
    for (uint64_t r = 0; r < 2 * rows; ++r)
        if (!(lam[r] > 0.0) || !std::isfinite(lam[r]))
            return fail(PPS_EINVAL, "lambda[%llu] must be finite and > 0",
                        static_cast<unsigned long long>(r));
    return PPS_OK;
}

// Persistent grid of the SMC kernel, zeroed tile counter, timed launch.
int run_smc(Context &c, const BioDesign &b, const SmcParams &p, uint64_t seed, SmcRuns runs,
            hipStream_t stream)
{
    hipError_t e = c.smc_ctr.ensure(256);
    if (e != hipSuccess)
        return fail_hip(e, "SMC tile counter");
    runs.next_run = c.smc_ctr.as<unsigned long long>();
    if ((e = hipMemsetAsync(runs.next_run, 0, sizeof(unsigned long long), stream)) != hipSuccess)
        return fail_hip(e, "SMC tile counter reset");
    const int block = smc_block_for(p.n_particles);
    int per_cu = 0;
    if (smc_occupancy(block, &per_cu) != hipSuccess || per_cu < 1)
        per_cu = 1;
    uint64_t grid = static_cast<uint64_t>(per_cu) * c.cu_count;
    if (grid > runs.n_runs)
        grid = runs.n_runs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_timing) {
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
        (void)hipEventRecord(ev0, stream);
    }
    e = launch_smc(b, p, seed, runs, static_cast<unsigned>(grid), stream);
    if (e != hipSuccess)
        return fail_hip(e, "SMC launch");
    if (g_timing) {
        (void)hipEventRecord(ev1, stream);
        float ms = -1.0f;
        if (hipEventSynchronize(ev1) == hipSuccess && hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess)
            c.last_kernel_ms = ms;
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    return PPS_OK;
}

}  // namespace

extern "C" {

int pps_smc_log_evidence(const pps_bioassay *model, const int32_t *y, const double *lambda,
                         uint64_t n_sets, const pps_smc_config *smc, uint64_t seed,
                         uint64_t first_run, double *log_z, void *stream)
{
    clear_error();
    BioDesign b;
    SmcParams p;
    int rc;
    if ((rc = validate_bio(model, &b)) != PPS_OK || (rc = validate_smc(smc, &p)) != PPS_OK)
        return rc;
    if (n_sets < 1 || n_sets > (1ull << 40) || !y || !log_z)
        return fail(PPS_EINVAL, "pps_smc_log_evidence: n_sets, y and log_z are required");
    if ((rc = check_lambdas(lambda, n_sets)) != PPS_OK)
        return rc;
    for (uint64_t s = 0; s < n_sets; ++s)
        for (int i = 0; i < b.n_groups; ++i)
            if (y[s * b.n_groups + i] < 0 || y[s * b.n_groups + i] > b.n_trials[i])
                return fail(PPS_EINVAL, "y[%llu][%d] outside [0, n_trials]",
                            static_cast<unsigned long long>(s), i);
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t ybytes = n_sets * b.n_groups * sizeof(int32_t);
    const size_t lbytes = n_sets * 2 * sizeof(double);
    // sum_i log C(n_i, y_i) of every set (the likelihood's constant)
    std::vector<double> lcoef(n_sets);
    for (uint64_t s = 0; s < n_sets; ++s) {
        double lc = 0.0;
        for (int i = 0; i < b.n_groups; ++i) {
            const double n = b.n_trials[i], k = y[s * b.n_groups + i];
            lc += std::lgamma(n + 1.0) - std::lgamma(k + 1.0) - std::lgamma(n - k + 1.0);
        }
        lcoef[s] = lc;
    }
    hipError_t e;
    if ((e = c->smc_y.ensure(ybytes)) != hipSuccess || (e = c->smc_lam.ensure(lbytes)) != hipSuccess ||
        (e = c->smc_coef.ensure(n_sets * sizeof(double))) != hipSuccess)
        return fail_hip(e, "SMC inputs");
    if ((e = hipMemcpyAsync(c->smc_y.p, y, ybytes, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(c->smc_lam.p, lambda, lbytes, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(c->smc_coef.p, lcoef.data(), n_sets * sizeof(double),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail_hip(e, "SMC input copy");
    // the host vectors must outlive the copies
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_hip(e, "SMC input copy");
    SmcRuns runs{};
    runs.mode = 0;
    runs.n_runs = n_sets;
    runs.first_run = first_run;
    runs.y = c->smc_y.as<int32_t>();
    runs.lam = c->smc_lam.as<double>();
    runs.lcoef = c->smc_coef.as<double>();
    runs.out0 = log_z;
    if ((rc = run_smc(*c, b, p, seed, runs, st)) != PPS_OK)
        return rc;
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_hip(e, "pps_smc_log_evidence");
    return PPS_OK;
}

int pps_wip_test(const pps_bioassay *model, const double *lambda, int n_lambda, uint64_t n_data,
                 const pps_smc_config *smc, uint64_t seed, double alpha, double *log_z0,
                 double *log_zk, double *pvalues, double *gamma, void *stream)
{
    clear_error();
    BioDesign b;
    SmcParams p;
    int rc;
    if ((rc = validate_bio(model, &b)) != PPS_OK || (rc = validate_smc(smc, &p)) != PPS_OK)
        return rc;
    if (n_lambda < 1 || n_lambda > 65536)
        return fail(PPS_EINVAL, "n_lambda %d out of range [1, 65536]", n_lambda);
    if (n_data < 1 || n_data > 65536)
        return fail(PPS_EINVAL, "n_data out of range [1, 65536]");
    if (!(alpha > 0.0 && alpha <= 1.0))
        return fail(PPS_EINVAL, "alpha must be in (0, 1]");
    if (!log_z0 || !log_zk || !gamma)
        return fail(PPS_EINVAL, "log_z0, log_zk and gamma are required");
    if ((rc = check_lambdas(lambda, static_cast<uint64_t>(n_lambda))) != PPS_OK)
        return rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t sets = n_data * (1 + static_cast<uint64_t>(n_lambda));
    const size_t ybytes = sets * b.n_groups * sizeof(int32_t);
    const size_t lbytes = static_cast<size_t>(n_lambda) * 2 * sizeof(double);
    const size_t cbytes = static_cast<size_t>(n_lambda) * n_data * sizeof(uint32_t);
    hipError_t e;
    if ((e = c->smc_y.ensure(ybytes)) != hipSuccess || (e = c->smc_lam.ensure(lbytes)) != hipSuccess ||
        (e = c->smc_counts.ensure(cbytes)) != hipSuccess ||
        (e = c->smc_gamma.ensure(n_lambda * sizeof(double))) != hipSuccess ||
        (e = c->smc_coef.ensure(sets * sizeof(double))) != hipSuccess)
        return fail_hip(e, "weak-informativity scratch");
    if ((e = hipMemcpyAsync(c->smc_lam.p, lambda, lbytes, hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail_hip(e, "lambda copy");
    int32_t *y0 = c->smc_y.as<int32_t>();
    int32_t *yk = y0 + n_data * b.n_groups;
    if ((e = launch_bio_data(b, c->smc_lam.as<double>(), n_lambda, n_data, seed, y0, yk,
                             c->smc_coef.as<double>(), st)) != hipSuccess)
        return fail_hip(e, "data-set launch");
    SmcRuns runs{};
    runs.mode = 1;
    runs.n_runs = 2 * static_cast<uint64_t>(n_lambda) * n_data;
    runs.n_data = n_data;
    runs.y = y0;
    runs.yk = yk;
    runs.lam = c->smc_lam.as<double>();
    runs.lcoef = c->smc_coef.as<double>();
    runs.out0 = log_z0;
    runs.outk = log_zk;
    if ((rc = run_smc(*c, b, p, seed, runs, st)) != PPS_OK)
        return rc;
    uint64_t q = static_cast<uint64_t>(std::ceil(alpha * static_cast<double>(n_data)));
    q = q < 1 ? 1 : (q > n_data ? n_data : q);
    if ((e = launch_wip_tally(log_z0, log_zk, n_lambda, n_data, q, c->smc_counts.as<uint32_t>(),
                              pvalues, c->smc_gamma.as<double>(), st)) != hipSuccess)
        return fail_hip(e, "tally launch");
    if ((e = hipMemcpyAsync(gamma, c->smc_gamma.p, n_lambda * sizeof(double), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return fail_hip(e, "pps_wip_test");
    return PPS_OK;
}

}  // extern "C"
