// extern "C" entry point of the BEGE log-likelihood (declared in
// include/pps.h): validation, scratch and the launches of pps_bege.hip.
#include "pps.h"
#include "pps_bege.hpp"
#include "pps_runtime.hpp"

using namespace pps;

namespace {

int bege_run(const double *theta, int n_theta, const double *r, int T, int n_omega, double *loglik,
             double *logdens, double *ops_host, void *stream)
{
    if (n_theta < 1 || n_theta > PPS_BEGE_MAX_THETA)
        return fail(PPS_EINVAL, "n_theta %d out of range [1, %d]", n_theta, PPS_BEGE_MAX_THETA);
    if (T < 1 || T > PPS_BEGE_MAX_T)
        return fail(PPS_EINVAL, "T %d out of range [1, %d]", T, PPS_BEGE_MAX_T);
    if (static_cast<uint64_t>(n_theta) * static_cast<uint64_t>(T) > PPS_BEGE_MAX_CELLS)
        return fail(PPS_EINVAL, "n_theta * T exceeds %llu",
                    static_cast<unsigned long long>(PPS_BEGE_MAX_CELLS));
    if (n_omega < 2 || n_omega > PPS_BEGE_MAX_NODES)
        return fail(PPS_EINVAL, "n_omega %d out of range [2, %d]", n_omega, PPS_BEGE_MAX_NODES);
    if (!theta || !r || (!loglik && !ops_host))
        return fail(PPS_EINVAL, "theta, r and loglik are required");
    int rc;
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t cells = static_cast<size_t>(n_theta) * T;
    hipError_t e;
    // shapes, the operation total, chunk classes and order; per-step log
    // densities and sums when the caller does not take them
    const int chunks = bege_chunks(T);
    const size_t n_chunks = static_cast<size_t>(n_theta) * chunks;
    if ((e = c->bege_shapes.ensure(2 * cells * sizeof(double) + 256 + 2 * n_chunks * sizeof(int32_t))) !=
            hipSuccess ||
        (!logdens && (e = c->bege_logdens.ensure((cells + n_theta) * sizeof(double))) != hipSuccess))
        return fail_hip(e, "BEGE scratch");
    BegeBatch b{};
    b.theta = theta;
    b.r = r;
    b.n_theta = n_theta;
    b.T = T;
    b.n_omega = n_omega;
    b.chunks = chunks;
    b.shape_p = c->bege_shapes.as<double>();
    b.shape_n = b.shape_p + cells;
    // after the shapes: the operation total (256 bytes), then the chunk
    // classes and order
    b.chunk_class = reinterpret_cast<int32_t *>(b.shape_n + cells + 32);
    b.chunk_order = b.chunk_class + n_chunks;
    b.logdens = logdens ? logdens : c->bege_logdens.as<double>();
    b.loglik = loglik ? loglik : c->bege_logdens.as<double>() + cells;
    if (ops_host) {
        // the operation total sits after the shapes
        b.ops = b.shape_n + cells;
        if ((e = hipMemsetAsync(b.ops, 0, sizeof(double), st)) != hipSuccess)
            return fail_hip(e, "BEGE operation counter");
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_timing) {
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
    }
    e = launch_bege(b, st, ev0, ev1);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (g_timing) {
        float ms = -1.0f;
        if (e == hipSuccess && hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess)
            c->last_kernel_ms = ms;
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    if (e == hipSuccess && ops_host)
        e = hipMemcpy(ops_host, b.ops, sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e, "BEGE launch");
    return PPS_OK;
}

}  // namespace

extern "C" {

int pps_bege_loglik(const double *theta, int n_theta, const double *r, int T, int n_omega,
                    double *loglik, double *logdens, void *stream)
{
    clear_error();
    return bege_run(theta, n_theta, r, T, n_omega, loglik, logdens, nullptr, stream);
}

int pps_bege_count_ops(const double *theta, int n_theta, const double *r, int T, int n_omega,
                       double *ops, void *stream)
{
    clear_error();
    if (!ops)
        return fail(PPS_EINVAL, "ops is required");
    return bege_run(theta, n_theta, r, T, n_omega, nullptr, nullptr, ops, stream);
}

}  // extern "C"
