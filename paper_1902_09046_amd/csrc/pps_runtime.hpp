// Host runtime of libpps: per-device context, buffers, job-table launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "pps.h"
#include "pps_internal.hpp"

namespace pps {

// Records a message for pps_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);
int fail_hip(hipError_t e, const char *what);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    template <class T> T *as() const { return static_cast<T *>(p); }
};

struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Launch shape of the simulation kernel for one model class.
struct LaunchShape {
    int block = 256;
};

struct Context {
    int device = -1;
    int cu_count = 0;
    std::mutex mu;
    LaunchShape shape[2];
    int occupancy[2][4] = {{0}};  // blocks per CU for block sizes 64,128,256,512
    // device scratch
    DevBuf jobs, state, fins, results, dist, block_counts, partials, hist, counts;
    // pinned staging
    HostBuf h_jobs, h_fins, h_results, h_counts;
    // kernel timing (see pps_set_timing)
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool ev_pending = false;
    double last_kernel_ms = -1.0;
};

extern bool g_timing;
// After a synchronous call's final stream synchronisation: reads the event
// pair recorded around the simulation kernel, if any.
void collect_timing(Context &c);

// Context of the current HIP device (created on first use).
Context *current_context(int *status);

int model_class(const pps_model *m);
// Validates a model; on success returns PPS_OK and its summary count.
int validate_model(const pps_model *m, int *n_summ);
int validate_sampling(const pps_sampling *s);

// Fills a job row (no tiling, no outputs).
void fill_job(JobDev &J, const pps_model *m, const pps_sampling *s, int n_summ, int flags);

// Assigns tiles to rows (tile size = block), stages the table and launches
// the persistent simulation kernel of class `cls` on `stream`.
int launch_rows(Context &c, int cls, std::vector<JobDev> &rows, hipStream_t stream);

int blocks_per_cu(Context &c, int cls, int block);

uint64_t top_count(double frac, uint64_t n);

}  // namespace pps
