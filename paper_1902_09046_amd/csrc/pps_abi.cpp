// extern "C" entry points of libpps (declared in include/pps.h).
#include <cmath>
#include <cstring>
#include <vector>

#include "pps.h"
#include "pps_launch.hpp"
#include "pps_runtime.hpp"

namespace pps {
const char *last_error();
void clear_error();
}  // namespace pps

using namespace pps;

#define PPS_TRY_HIP(expr, what)                                                                \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail_hip(e_, what);                                                         \
    } while (0)

static hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

extern "C" {

const char *pps_version(void) { return "pps 0.1 (gfx950)"; }

const char *pps_last_error(void) { return last_error(); }

int pps_set_timing(int enable)
{
    g_timing = enable != 0;
    return PPS_OK;
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
    if (model_class != CLASS_PATH && model_class != CLASS_GARCH)
        return fail(PPS_EINVAL, "unknown model class %d", model_class);
    if (block != 64 && block != 128 && block != 256 && block != 512)
        return fail(PPS_EINVAL, "block size %d not in {64, 128, 256, 512}", block);
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    c->shape[model_class].block = block;
    return PPS_OK;
}

int pps_get_block_size(int model_class)
{
    clear_error();
    if (model_class != CLASS_PATH && model_class != CLASS_GARCH)
        return fail(PPS_EINVAL, "unknown model class %d", model_class);
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    return c->shape[model_class].block;
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
    if ((rc = validate_model(model, &ns)) != PPS_OK)
        return rc;
    if ((rc = validate_sampling(sampling)) != PPS_OK)
        return rc;
    if (dist && !y_obs)
        return fail(PPS_EINVAL, "pps_simulate: dist requested without y_obs");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    std::vector<JobDev> rows(1);
    fill_job(rows[0], model, sampling, ns, JOB_DUMP);
    JobDev &J = rows[0];
    if (y_obs && model->model != PPS_GARCH11)
        for (int k = 0; k < ns; ++k)
            J.y_obs[k] = static_cast<float>(y_obs[k]);
    J.dump_theta = theta;
    J.dump_summ = summ;
    J.dump_stat = model->model == PPS_GARCH11 ? nullptr : stat;
    J.dump_dist = model->model == PPS_GARCH11 ? nullptr : dist;
    const hipStream_t s = as_stream(stream);
    if ((rc = launch_rows(*c, model_class(model), rows, s)) != PPS_OK)
        return rc;
    PPS_TRY_HIP(hipStreamSynchronize(s), "pps_simulate");
    collect_timing(*c);
    return PPS_OK;
}

int abc_sample(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
               int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
               float *acc_theta, float *acc_dist, pps_abc_stats *stats, void *stream)
{
    clear_error();
    int ns = 0, rc;
    if ((rc = validate_model(model, &ns)) != PPS_OK)
        return rc;
    if ((rc = validate_sampling(sampling)) != PPS_OK)
        return rc;
    if (model->model == PPS_GARCH11)
        return fail(PPS_EINVAL, "abc_sample: GARCH summaries have no observed-data distance here");
    if (!y_obs || !stats)
        return fail(PPS_EINVAL, "abc_sample: y_obs and stats are required");
    if (eps_mode != PPS_EPS_FIXED && eps_mode != PPS_EPS_TOP_FRACTION)
        return fail(PPS_EINVAL, "abc_sample: unknown eps_mode %d", eps_mode);
    if (eps_mode == PPS_EPS_TOP_FRACTION && !(eps_or_frac > 0.0 && eps_or_frac <= 1.0))
        return fail(PPS_EINVAL, "abc_sample: fraction must be in (0, 1]");
    if (eps_mode == PPS_EPS_FIXED && std::isnan(eps_or_frac))
        return fail(PPS_EINVAL, "abc_sample: eps is NaN");
    if (capacity > 0 && (!acc_idx || !acc_theta || !acc_dist))
        return fail(PPS_EINVAL, "abc_sample: output buffers required when capacity > 0");
    if (sampling->n_draws >= (1ull << 32))
        return fail(PPS_EINVAL, "abc_sample: n_draws must be < 2^32");
    for (int k = 0; k < ns; ++k)
        if (!std::isfinite(y_obs[k]))
            return fail(PPS_EINVAL, "abc_sample: y_obs[%d] is not finite", k);
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    const uint64_t n = sampling->n_draws;
    const uint64_t nb = (n + FIN_TILE - 1) / FIN_TILE;
    PPS_TRY_HIP(c->dist.ensure(n * sizeof(float)), "distance buffer");
    PPS_TRY_HIP(c->fins.ensure(sizeof(FinJob)), "finalisation table");
    PPS_TRY_HIP(c->results.ensure(sizeof(FinResult)), "result row");
    PPS_TRY_HIP(c->hist.ensure(SEL_BINS * sizeof(unsigned)), "select histogram");
    PPS_TRY_HIP(c->block_counts.ensure(2 * nb * sizeof(unsigned long long)), "block counts");
    PPS_TRY_HIP(c->partials.ensure(nb * (1 + 2 * PPS_MAX_PARAMS) * sizeof(double)), "partials");
    PPS_TRY_HIP(c->h_fins.ensure(sizeof(FinJob)), "pinned staging");
    PPS_TRY_HIP(c->h_results.ensure(sizeof(FinResult)), "pinned staging");

    std::vector<JobDev> rows(1);
    fill_job(rows[0], model, sampling, ns, JOB_WRITE_DIST);
    for (int k = 0; k < ns; ++k)
        rows[0].y_obs[k] = static_cast<float>(y_obs[k]);
    rows[0].dist = c->dist.as<float>();
    const hipStream_t s = as_stream(stream);
    if ((rc = launch_rows(*c, CLASS_PATH, rows, s)) != PPS_OK)
        return rc;

    FinJob F;
    std::memset(&F, 0, sizeof F);
    F.dist = c->dist.as<float>();
    F.n = n;
    F.first_draw = sampling->first_draw;
    F.seed = sampling->seed;
    F.mode = eps_mode;
    F.n_params = model->n_params;
    F.constraint = model->constraint;
    F.eps = eps_mode == PPS_EPS_FIXED ? eps_or_frac : 0.0;
    F.k = eps_mode == PPS_EPS_TOP_FRACTION ? top_count(eps_or_frac, n) : 0;
    F.capacity = capacity;
    F.block_begin = 0;
    F.n_blocks = nb;
    std::memcpy(F.prior, rows[0].prior, sizeof F.prior);
    F.acc_idx = acc_idx;
    F.acc_theta = acc_theta;
    F.acc_dist = acc_dist;
    F.hist = c->hist.as<unsigned>();
    F.block_counts = c->block_counts.as<unsigned long long>();
    F.partials = c->partials.as<double>();
    F.result = c->results.as<FinResult>();
    std::memcpy(c->h_fins.p, &F, sizeof F);
    PPS_TRY_HIP(hipMemcpyAsync(c->fins.p, c->h_fins.p, sizeof F, hipMemcpyHostToDevice, s),
                "finalisation upload");
    PPS_TRY_HIP(launch_abc_finalize(c->fins.as<FinJob>(), 1, nb,
                                    eps_mode == PPS_EPS_TOP_FRACTION, s),
                "finalisation launch");
    PPS_TRY_HIP(hipMemcpyAsync(c->h_results.p, c->results.p, sizeof(FinResult),
                               hipMemcpyDeviceToHost, s),
                "result download");
    PPS_TRY_HIP(hipStreamSynchronize(s), "abc_sample");
    collect_timing(*c);
    const FinResult *R = c->h_results.as<FinResult>();
    stats->n_accepted = R->n_accepted;
    stats->eps_used = R->eps_used;
    for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
        stats->mean[j] = R->mean[j];
        stats->var[j] = R->var[j];
    }
    if (R->n_accepted > capacity)
        return fail(PPS_ETRUNC, "abc_sample: %llu accepted, capacity %llu",
                    static_cast<unsigned long long>(R->n_accepted),
                    static_cast<unsigned long long>(capacity));
    return PPS_OK;
}

int prior_pred_pvalue(const pps_model *model, int lambda_param, int lambda_family,
                      const double *lambda, int n_lambda, const pps_sampling *sampling,
                      double t_obs, uint64_t *count_ge, double *pvalue, void *stream)
{
    clear_error();
    int ns = 0, rc;
    if ((rc = validate_model(model, &ns)) != PPS_OK)
        return rc;
    if ((rc = validate_sampling(sampling)) != PPS_OK)
        return rc;
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
    std::vector<JobDev> rows(n_lambda);
    for (int k = 0; k < n_lambda; ++k) {
        pps_model mk = *model;
        mk.prior[lambda_param].family = lambda_family;
        mk.prior[lambda_param].b = lambda[k];
        int ns2 = 0;
        if ((rc = validate_model(&mk, &ns2)) != PPS_OK)
            return fail(PPS_EINVAL, "lambda[%d] = %g gives an invalid prior", k, lambda[k]);
        fill_job(rows[k], &mk, sampling, ns, JOB_TALLY_STAT);
        rows[k].t_obs = t_obs;
        rows[k].lambda_group = 0;
    }
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    PPS_TRY_HIP(c->counts.ensure(n_lambda * sizeof(unsigned long long)), "tally buffer");
    PPS_TRY_HIP(c->h_counts.ensure(n_lambda * sizeof(unsigned long long)), "pinned staging");
    for (int k = 0; k < n_lambda; ++k)
        rows[k].counts = c->counts.as<unsigned long long>() + k;
    const hipStream_t s = as_stream(stream);
    PPS_TRY_HIP(launch_fill_u64(c->counts.as<unsigned long long>(), n_lambda, 0ull, s), "tally reset");
    if ((rc = launch_rows(*c, CLASS_PATH, rows, s)) != PPS_OK)
        return rc;
    PPS_TRY_HIP(hipMemcpyAsync(c->h_counts.p, c->counts.p, n_lambda * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s),
                "tally download");
    PPS_TRY_HIP(hipStreamSynchronize(s), "prior_pred_pvalue");
    collect_timing(*c);
    const unsigned long long *cnt = c->h_counts.as<unsigned long long>();
    for (int k = 0; k < n_lambda; ++k) {
        count_ge[k] = cnt[k];
        pvalue[k] = static_cast<double>(cnt[k]) / static_cast<double>(sampling->n_draws);
    }
    return PPS_OK;
}

int pps_summary_tally(const pps_model *model, const pps_sampling *sampling,
                      const double *obs_summ, uint64_t *count_ge, void *stream)
{
    clear_error();
    int ns = 0, rc;
    if ((rc = validate_model(model, &ns)) != PPS_OK)
        return rc;
    if ((rc = validate_sampling(sampling)) != PPS_OK)
        return rc;
    if (model->model != PPS_GARCH11)
        return fail(PPS_EINVAL, "pps_summary_tally: GARCH models only");
    if (!obs_summ || !count_ge)
        return fail(PPS_EINVAL, "obs_summ and count_ge are required");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    PPS_TRY_HIP(c->counts.ensure(ns * sizeof(unsigned long long)), "tally buffer");
    PPS_TRY_HIP(c->h_counts.ensure(ns * sizeof(unsigned long long)), "pinned staging");
    std::vector<JobDev> rows(1);
    fill_job(rows[0], model, sampling, ns, JOB_TALLY_SUMM);
    for (int k = 0; k < ns; ++k)
        rows[0].summ_obs[k] = obs_summ[k];
    rows[0].counts = c->counts.as<unsigned long long>();
    const hipStream_t s = as_stream(stream);
    PPS_TRY_HIP(launch_fill_u64(c->counts.as<unsigned long long>(), ns, 0ull, s), "tally reset");
    if ((rc = launch_rows(*c, CLASS_GARCH, rows, s)) != PPS_OK)
        return rc;
    PPS_TRY_HIP(hipMemcpyAsync(c->h_counts.p, c->counts.p, ns * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s),
                "tally download");
    PPS_TRY_HIP(hipStreamSynchronize(s), "pps_summary_tally");
    collect_timing(*c);
    std::memcpy(count_ge, c->h_counts.p, ns * sizeof(unsigned long long));
    return PPS_OK;
}

}  // extern "C"
