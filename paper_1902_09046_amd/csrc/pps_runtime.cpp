// Host runtime of libpps: errors, per-device contexts, buffers, validation
// and job-table launches of the persistent simulation kernel.
#include "pps_runtime.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "pps_launch.hpp"

namespace pps {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? PPS_ENOMEM : PPS_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

const char *last_error() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

hipError_t DevBuf::ensure(size_t need)
{
    if (need <= bytes && p)
        return hipSuccess;
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        bytes = 0;
        if (e != hipSuccess)
            return e;
    }
    size_t grow = need < 4096 ? 4096 : need + need / 4;
    hipError_t e = hipMalloc(&p, grow);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return e;
    }
    bytes = grow;
    return hipSuccess;
}

static constexpr int kMaxDevices = 64;
static Context *g_contexts[kMaxDevices];
static std::mutex g_contexts_mu;

Context *current_context(int *status)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *status = fail_hip(e, "hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *status = fail(PPS_EDEVICE, "device %d out of range", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_contexts_mu);
    if (!g_contexts[dev]) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) {
            *status = fail_hip(e, "hipGetDeviceProperties");
            return nullptr;
        }
        Context *c = new Context();
        c->device = dev;
        c->cu_count = prop.multiProcessorCount;
        for (auto &r : c->noalloc_plan.rows)
            r.reserve(1);
        c->noalloc_plan.fins.reserve(1);
        c->engine.reset(new EpochEngine());
        int rc = c->engine->init(1, c->cu_count);
        if (rc != PPS_OK) {
            *status = rc;
            return nullptr;  // the partially built context is leaked on purpose
        }
        g_contexts[dev] = c;
    }
    *status = PPS_OK;
    return g_contexts[dev];
}

Context *existing_context(int *status)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *status = fail_hip(e, "hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *status = fail(PPS_EDEVICE, "device %d out of range", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_contexts_mu);
    if (!g_contexts[dev]) {
        *status = fail(PPS_EINVAL, "device %d has no context yet (any other call creates it)", dev);
        return nullptr;
    }
    *status = PPS_OK;
    return g_contexts[dev];
}

int model_class(const pps_model *m)
{
    if (m->model == PPS_GARCH11)
        return CLASS_GARCH;
    if (m->model == PPS_TOGGLE_SWITCH)
        return CLASS_CELLS;
    if (m->model == PPS_TB)
        return CLASS_GILLESPIE;
    return CLASS_PATH;
}

static bool finite(double v) { return std::isfinite(v); }

int validate_model(const pps_model *m, int *n_summ)
{
    if (!m)
        return fail(PPS_EINVAL, "model is NULL");
    if (m->n_params < 1 || m->n_params > PPS_MAX_PARAMS)
        return fail(PPS_EINVAL, "n_params %d out of range [1, %d]", m->n_params, PPS_MAX_PARAMS);
    for (int j = 0; j < m->n_params; ++j) {
        const pps_prior &p = m->prior[j];
        switch (p.family) {
        case PPS_UNIFORM:
            if (!finite(p.a) || !finite(p.b) || !(p.a < p.b))
                return fail(PPS_EINVAL, "prior %d: uniform needs finite a < b", j);
            break;
        case PPS_NORMAL:
        case PPS_LOGNORMAL:
            if (!finite(p.a) || !finite(p.b) || p.b < 0.0)
                return fail(PPS_EINVAL, "prior %d: (log)normal needs finite mean and sd >= 0", j);
            break;
        case PPS_POINT:
            if (std::isnan(p.a))
                return fail(PPS_EINVAL, "prior %d: point mass at NaN", j);
            break;
        default:
            return fail(PPS_EINVAL, "prior %d: unknown family %d", j, p.family);
        }
    }
    if (m->constraint != PPS_NO_CONSTRAINT && m->constraint != PPS_GARCH_STATIONARY &&
        m->constraint != PPS_TB_SUPERCRITICAL)
        return fail(PPS_EINVAL, "unknown constraint %d", m->constraint);
    if (m->constraint == PPS_TB_SUPERCRITICAL && m->model != PPS_TB)
        return fail(PPS_EINVAL, "the supercritical constraint only applies to tuberculosis");
    switch (m->model) {
    case PPS_LOGISTIC_SDE:
        if (m->n_params != 3)
            return fail(PPS_EINVAL, "logistic SDE needs 3 parameters");
        if (m->n_obs < 1 || m->n_obs > PPS_MAX_OBS)
            return fail(PPS_EINVAL, "n_obs %d out of range [1, %d]", m->n_obs, PPS_MAX_OBS);
        if (m->steps < 1 || m->steps % m->n_obs != 0)
            return fail(PPS_EINVAL, "steps %d must be a positive multiple of n_obs %d", m->steps,
                        m->n_obs);
        if (!finite(m->t_end) || !(m->t_end > 0.0) || !finite(m->x0))
            return fail(PPS_EINVAL, "logistic SDE needs finite t_end > 0 and x0");
        if (m->constraint != PPS_NO_CONSTRAINT)
            return fail(PPS_EINVAL, "constraint only applies to GARCH");
        *n_summ = m->n_obs;
        return PPS_OK;
    case PPS_NORMAL_MEAN:
        if (m->n_obs < 1 || m->n_obs > PPS_MAX_OBS)
            return fail(PPS_EINVAL, "n_obs %d out of range [1, %d]", m->n_obs, PPS_MAX_OBS);
        if (!finite(m->noise_sd) || m->noise_sd < 0.0)
            return fail(PPS_EINVAL, "noise_sd must be finite and >= 0");
        if (m->constraint != PPS_NO_CONSTRAINT)
            return fail(PPS_EINVAL, "constraint only applies to GARCH");
        *n_summ = m->n_obs;
        return PPS_OK;
    case PPS_GARCH11:
        if (m->n_params != 3)
            return fail(PPS_EINVAL, "GARCH needs 3 parameters (omega, alpha, beta)");
        if (m->steps < 20 || m->steps % 20 != 0)
            return fail(PPS_EINVAL, "GARCH series length %d must be a positive multiple of 20",
                        m->steps);
        *n_summ = PPS_GARCH_NSUMM;
        return PPS_OK;
    case PPS_TOGGLE_SWITCH:
        if (m->n_params != 7)
            return fail(PPS_EINVAL, "toggle switch needs 7 parameters "
                                    "(mu, sigma, gamma, alpha_u, alpha_v, beta_u, beta_v)");
        if (m->n_cells < 1 || m->n_cells > PPS_TSW_MAX_CELLS)
            return fail(PPS_EINVAL, "n_cells %d out of range [1, %d]", m->n_cells,
                        PPS_TSW_MAX_CELLS);
        if (m->n_obs < 1 || m->n_obs > PPS_MAX_OBS)
            return fail(PPS_EINVAL, "n_obs (quantiles) %d out of range [1, %d]", m->n_obs,
                        PPS_MAX_OBS);
        if (m->steps < 1)
            return fail(PPS_EINVAL, "toggle switch needs steps >= 1");
        if (!finite(m->t_end) || !(m->t_end > 0.0) || !finite(m->x0))
            return fail(PPS_EINVAL, "toggle switch needs finite t_end > 0 and x0");
        if (m->constraint != PPS_NO_CONSTRAINT)
            return fail(PPS_EINVAL, "constraint only applies to GARCH");
        *n_summ = m->n_obs;
        return PPS_OK;
    case PPS_TB:
        if (m->n_params != 3)
            return fail(PPS_EINVAL, "tuberculosis needs 3 parameters (alpha, delta, tau)");
        if (m->n_cells < 2 || m->n_cells > PPS_TB_MAX_POP)
            return fail(PPS_EINVAL, "stopping population %d out of range [2, %d]", m->n_cells,
                        PPS_TB_MAX_POP);
        if (m->n_obs < 1 || m->n_obs > PPS_TB_MAX_SAMPLE)
            return fail(PPS_EINVAL, "sample size %d out of range [1, %d]", m->n_obs,
                        PPS_TB_MAX_SAMPLE);
        if (m->steps < 1)
            return fail(PPS_EINVAL, "tuberculosis needs an event cap (steps) >= 1");
        if (!(m->x0 >= 1.0) || !(m->x0 <= m->n_cells) || m->x0 != std::floor(m->x0))
            return fail(PPS_EINVAL, "initial cases x0 must be an integer in [1, n_cells]");
        if (m->constraint == PPS_GARCH_STATIONARY)
            return fail(PPS_EINVAL, "the GARCH constraint does not apply to tuberculosis");
        *n_summ = 2;
        return PPS_OK;
    default:
        return fail(PPS_EINVAL, "unknown model %d", m->model);
    }
}

int validate_sampling(const pps_sampling *s)
{
    if (!s)
        return fail(PPS_EINVAL, "sampling is NULL");
    if (s->n_draws == 0)
        return fail(PPS_EINVAL, "n_draws must be >= 1");
    if (s->first_draw + s->n_draws < s->first_draw)
        return fail(PPS_EINVAL, "draw range overflows 64 bits");
    return PPS_OK;
}

void fill_job(JobDev &J, const pps_model *m, const pps_sampling *s, int n_summ, int flags)
{
    std::memset(&J, 0, sizeof J);
    J.model = m->model;
    J.flags = flags;
    J.n_params = m->n_params;
    J.n_summ = n_summ;
    J.constraint = m->constraint;
    if (m->model == PPS_LOGISTIC_SDE) {
        J.steps = m->steps;
        J.obs_stride = m->steps / m->n_obs;
        J.dt = m->t_end / static_cast<double>(m->steps);
    } else if (m->model == PPS_GARCH11) {
        J.steps = m->steps;
        J.obs_stride = 1;
    } else if (m->model == PPS_TOGGLE_SWITCH) {
        J.steps = m->steps;
        J.obs_stride = 1;
        J.dt = m->t_end / static_cast<double>(m->steps);
        J.n_cells = m->n_cells;
    } else if (m->model == PPS_TB) {
        J.steps = m->steps;
        J.obs_stride = 1;
        J.n_cells = m->n_cells;
        J.n_sample = m->n_obs;
    } else {
        J.steps = m->n_obs;
        J.obs_stride = 1;
    }
    J.seed = s->seed;
    J.first_draw = s->first_draw;
    J.n_draws = s->n_draws;
    for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
        J.prior[j].family = j < m->n_params ? m->prior[j].family : PPS_POINT;
        J.prior[j].a = j < m->n_params ? m->prior[j].a : 0.0;
        J.prior[j].b = j < m->n_params ? m->prior[j].b : 0.0;
    }
    J.x0 = m->x0;
    J.noise_sd = m->noise_sd;
}

bool g_timing = false;

static size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

size_t abc_scratch_bytes(uint64_t n) { return abc_scratch_bound(n); }

AbcScratch abc_scratch_at(void *base, uint64_t n)
{
    const uint64_t nb = (n + FIN_TILE - 1) / FIN_TILE;
    char *p = static_cast<char *>(base);
    AbcScratch s;
    s.dist = reinterpret_cast<float *>(p);
    p += align256(n * sizeof(float));
    s.block_counts = reinterpret_cast<unsigned long long *>(p);
    p += align256(2 * nb * sizeof(unsigned long long));
    s.partials = reinterpret_cast<double *>(p);
    p += align256(nb * (1 + 2 * PPS_MAX_PARAMS) * sizeof(double));
    s.hist = reinterpret_cast<unsigned *>(p);
    p += align256(SEL_BINS * sizeof(unsigned));
    s.result = reinterpret_cast<FinResult *>(p);
    return s;
}

int validate_abc(const pps_model *m, const double *y_obs, int n_summ, const pps_sampling *s,
                 int eps_mode, double eps_or_frac)
{
    if (m->model == PPS_GARCH11)
        return fail(PPS_EINVAL, "ABC: GARCH summaries have no observed-data distance here");
    if (!y_obs)
        return fail(PPS_EINVAL, "ABC: y_obs is required");
    if (eps_mode != PPS_EPS_FIXED && eps_mode != PPS_EPS_TOP_FRACTION)
        return fail(PPS_EINVAL, "ABC: unknown eps_mode %d", eps_mode);
    if (eps_mode == PPS_EPS_TOP_FRACTION && !(eps_or_frac > 0.0 && eps_or_frac <= 1.0))
        return fail(PPS_EINVAL, "ABC: fraction must be in (0, 1]");
    if (eps_mode == PPS_EPS_FIXED && std::isnan(eps_or_frac))
        return fail(PPS_EINVAL, "ABC: eps is NaN");
    if (s->n_draws >= (1ull << 32))
        return fail(PPS_EINVAL, "ABC: n_draws must be < 2^32");
    for (int k = 0; k < n_summ; ++k)
        if (!std::isfinite(y_obs[k]))
            return fail(PPS_EINVAL, "ABC: y_obs[%d] is not finite", k);
    return PPS_OK;
}

void fill_fin(FinJob &F, const JobDev &row, int eps_mode, double eps_or_frac, uint64_t capacity,
              uint64_t *acc_idx, float *acc_theta, float *acc_dist, const AbcScratch &scr)
{
    std::memset(&F, 0, sizeof F);
    F.dist = scr.dist;
    F.n = row.n_draws;
    F.first_draw = row.first_draw;
    F.seed = row.seed;
    F.mode = eps_mode;
    F.n_params = row.n_params;
    F.constraint = row.constraint;
    F.eps = eps_mode == PPS_EPS_FIXED ? eps_or_frac : 0.0;
    F.k = eps_mode == PPS_EPS_TOP_FRACTION ? top_count(eps_or_frac, row.n_draws) : 0;
    F.capacity = capacity;
    std::memcpy(F.prior, row.prior, sizeof F.prior);
    F.acc_idx = acc_idx;
    F.acc_theta = acc_theta;
    F.acc_dist = acc_dist;
    F.hist = scr.hist;
    F.block_counts = scr.block_counts;
    F.partials = scr.partials;
    F.result = scr.result;
}

uint64_t top_count(double frac, uint64_t n)
{
    double k = std::ceil(frac * static_cast<double>(n));
    if (k < 1.0)
        k = 1.0;
    if (k > static_cast<double>(n))
        k = static_cast<double>(n);
    return static_cast<uint64_t>(k);
}

}  // namespace pps
