// Host-callable launchers for the kernels in pps_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pps_internal.hpp"

namespace pps {

// Resets the launch state, then runs the persistent simulation kernel over
// tiles [0, total_tiles) of the job table with `grid` workgroups of `block`.
// cls: CLASS_PATH (logistic, normal-mean) or CLASS_GARCH; every job in the
// table must belong to that class.
// When ev_start / ev_stop are not null they are recorded on `s` right
// before and after the simulation kernel (after the state reset).
hipError_t launch_simulate(int cls, int block, const JobDev *jobs, int n_jobs, uint64_t total_tiles,
                           LaunchState *state, unsigned grid, hipStream_t s,
                           hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t simulate_occupancy(int cls, int block, int *blocks_per_cu);

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_philox(uint64_t seed, uint64_t first, uint64_t n, uint32_t block,
                         uint32_t purpose, uint32_t *out, hipStream_t s);
hipError_t launch_normals(uint64_t seed, uint64_t first, uint64_t n, uint32_t m, float *out,
                          hipStream_t s);

// Select (top-fraction jobs), ordered compaction and moments for n_fins
// ABC jobs whose finalisation blocks span [0, total_blocks).
hipError_t launch_abc_finalize(const FinJob *fins, int n_fins, uint64_t total_blocks,
                               bool any_top, hipStream_t s);

}  // namespace pps
