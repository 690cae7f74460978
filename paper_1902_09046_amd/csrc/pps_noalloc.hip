// abc_sample_noalloc: the ABC call of abc_sample with its device scratch
// (distances, compaction block counts, moment partials, selection histogram,
// result) in a file-scope device array instead of memory the library
// allocates, for callers that cannot allocate.  The kernels, the epoch graph
// and the results are abc_sample's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pps.h"
#include "pps_runtime.hpp"

namespace pps {

// Largest prior sample one call may use, and the scratch it needs (16.2 MiB).
constexpr uint64_t NOALLOC_MAX_DRAWS = PPS_NOALLOC_MAX_DRAWS;
constexpr size_t NOALLOC_SCRATCH_BYTES = abc_scratch_bound(NOALLOC_MAX_DRAWS);

// One copy per device, held until the process ends.  In host code this name
// is a stand-in, not a device address: kernels get the address looked up
// below.  `used` keeps the device compiler from dropping an array no kernel
// names.
static __device__ __align__(256) __attribute__((used)) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static constexpr int kMaxScratchDevices = 64;
static void *g_scratch_ptr[kMaxScratchDevices];
static std::mutex g_scratch_mu;

// Device address of the current device's copy of `scratch`, looked up once
// per device (the device must be current).
static int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(PPS_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(PPS_EDEVICE, "scratch array has no device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PPS_OK;
}

}  // namespace pps

using namespace pps;

extern "C" {

int abc_sample_noalloc(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
                       int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
                       float *acc_theta, float *acc_dist, pps_abc_stats *stats, void *stream)
{
    clear_error();
    int ns = 0;
    int rc = abc_check(model, y_obs, sampling, eps_mode, eps_or_frac, capacity, acc_idx,
                       acc_theta, acc_dist, stats, &ns);
    if (rc != PPS_OK)
        return rc;
    if (sampling->n_draws > NOALLOC_MAX_DRAWS)
        return fail(PPS_EINVAL, "abc_sample_noalloc: n_draws %llu above its maximum %llu",
                    static_cast<unsigned long long>(sampling->n_draws),
                    static_cast<unsigned long long>(NOALLOC_MAX_DRAWS));
    Context *c = existing_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    void *base = nullptr;
    if ((rc = scratch_address(c->device, &base)) != PPS_OK)
        return rc;
    return abc_run(*c, model, ns, y_obs, sampling, eps_mode, eps_or_frac, capacity, acc_idx,
                   acc_theta, acc_dist, stats, base, c->noalloc_plan, false,
                   static_cast<hipStream_t>(stream));
}

}  // extern "C"
