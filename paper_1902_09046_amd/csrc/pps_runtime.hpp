// Host runtime of libpps: errors, buffers, per-device context, validation,
// job-row and finalisation-row construction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pps.h"
#include "pps_engine.hpp"
#include "pps_internal.hpp"

namespace pps {

// Records a message for pps_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);
int fail_hip(hipError_t e, const char *what);
const char *last_error();
void clear_error();

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Per-device state of the synchronous entry points: their epoch engine (one
// slot) and the scratch their jobs use.
struct Context {
    int device = -1;
    int cu_count = 0;
    std::mutex mu;
    std::unique_ptr<EpochEngine> engine;        // synchronous calls (one slot)
    std::unique_ptr<EpochEngine> batch_engine;  // pps_run_batch (two slots)
    DevBuf dist, block_counts, partials, hist, results, counts;
    // weak-informativity test: data sets, hyperparameters, tile counter,
    // tally counts and cut-offs
    DevBuf smc_y, smc_lam, smc_coef, smc_ctr, smc_counts, smc_gamma;
    // BEGE log-likelihood: the shapes of every (vector, t), and the per-t
    // log densities when the caller does not take them
    DevBuf bege_shapes, bege_logdens;
    // the epoch plan of abc_sample_noalloc, its vectors reserved when the
    // context is created so that the call allocates no host memory either
    EpochPlan noalloc_plan;
    double last_kernel_ms = -1.0;
    double last_finalize_ms = -1.0;
};

extern bool g_timing;

// Context of the current HIP device (created on first use, engine included).
Context *current_context(int *status);
// The current device's context if it exists; else NULL with PPS_EINVAL
// (creates nothing).
Context *existing_context(int *status);

int model_class(const pps_model *m);
// Validates a model; on success returns PPS_OK and its summary count.
int validate_model(const pps_model *m, int *n_summ);
int validate_sampling(const pps_sampling *s);

// Fills a job row for the whole job (tiles assigned by the engine).
void fill_job(JobDev &J, const pps_model *m, const pps_sampling *s, int n_summ, int flags);

// Per-job device scratch of an ABC finalisation.
struct AbcScratch {
    float *dist = nullptr;                    // n floats
    unsigned long long *block_counts = nullptr;  // 2 * blocks
    double *partials = nullptr;               // blocks * (1 + 2 * PPS_MAX_PARAMS)
    unsigned *hist = nullptr;                 // SEL_BINS
    FinResult *result = nullptr;              // 1
};
constexpr size_t abc_scratch_bound(uint64_t n)
{
    const uint64_t nb = (n + FIN_TILE - 1) / FIN_TILE;
    return ((n * sizeof(float) + 255) & ~size_t(255)) +
           ((2 * nb * sizeof(unsigned long long) + 255) & ~size_t(255)) +
           ((nb * (1 + 2 * PPS_MAX_PARAMS) * sizeof(double) + 255) & ~size_t(255)) +
           ((SEL_BINS * sizeof(unsigned) + 255) & ~size_t(255)) +
           ((sizeof(FinResult) + 255) & ~size_t(255));
}
size_t abc_scratch_bytes(uint64_t n);
// Carves an AbcScratch out of `base` (abc_scratch_bytes(n) bytes, 256-aligned).
AbcScratch abc_scratch_at(void *base, uint64_t n);

// Validates the ABC arguments shared by abc_sample and the server.
int validate_abc(const pps_model *m, const double *y_obs, int n_summ, const pps_sampling *s,
                 int eps_mode, double eps_or_frac);
void fill_fin(FinJob &F, const JobDev &row, int eps_mode, double eps_or_frac, uint64_t capacity,
              uint64_t *acc_idx, float *acc_theta, float *acc_dist, const AbcScratch &scr);

uint64_t top_count(double frac, uint64_t n);

// The ABC job of abc_sample on validated arguments, context lock held: the
// simulation writes rho into the scratch at `scratch` (abc_scratch_bytes(n)
// bytes), the finalisation selects, compacts and reduces.  `plan` is cleared
// and refilled; build == false replays an existing epoch graph only.
int abc_run(Context &c, const pps_model *model, int n_summ, const double *y_obs,
            const pps_sampling *sampling, int eps_mode, double eps_or_frac, uint64_t capacity,
            uint64_t *acc_idx, float *acc_theta, float *acc_dist, pps_abc_stats *stats,
            void *scratch, EpochPlan &plan, bool build, hipStream_t stream);
// Argument checks of abc_sample; on success *n_summ is the summary count.
int abc_check(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
              int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
              float *acc_theta, float *acc_dist, const pps_abc_stats *stats, int *n_summ);

}  // namespace pps
