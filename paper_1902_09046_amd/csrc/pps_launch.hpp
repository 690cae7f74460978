// Host-callable launchers for the kernels in pps_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pps_internal.hpp"

namespace pps {

// Launch shape of one simulation class: workgroup size, draws per lane (the
// draws of a lane are simulated interleaved) and Philox blocks generated per
// loop trip.  Results never depend on the shape.
struct SimShape {
    int block = 256;
    int dpl = 1;
    int unroll = 1;
    bool operator==(const SimShape &o) const
    {
        return block == o.block && dpl == o.dpl && unroll == o.unroll;
    }
};

// Shape of one epoch: a simulation shape and resident grid per class, and the
// grid of the per-element finalisation kernels.
struct EpochShape {
    SimShape sim[N_CLASSES];
    unsigned sim_grid[N_CLASSES] = {};
    unsigned fin_grid = 0;
    bool operator==(const EpochShape &o) const
    {
        for (int c = 0; c < N_CLASSES; ++c)
            if (!(sim[c] == o.sim[c]) || sim_grid[c] != o.sim_grid[c])
                return false;
        return fin_grid == o.fin_grid;
    }
};

constexpr unsigned STAGE_GRID = 64;

// Device-visible addresses used by one epoch slot.  h_* point into mapped
// pinned host memory; d_* into device memory.
struct EpochDevPtrs {
    const EpochHeader *h_hdr = nullptr;
    const JobDev *h_rows = nullptr;
    const FinJob *h_fins = nullptr;
    FinResult *h_out_fin = nullptr;
    unsigned long long *h_out_counts = nullptr;
    EpochHeader *d_hdr = nullptr;
    JobDev *d_rows = nullptr;
    FinJob *d_fins = nullptr;
    LaunchState *states = nullptr;  // N_CLASSES
};

bool sim_shape_supported(int cls, const SimShape &sh);
hipError_t sim_occupancy(int cls, const SimShape &sh, int *blocks_per_cu);

// An epoch is issued as parts, in order, on one stream: stage-in; the
// simulation kernel of each class that has tiles; the ABC finalisation kernels
// (when the epoch finishes ABC jobs: EPOCH_FINALIZE with the tolerance
// selection passes when one of them takes the closest fraction,
// EPOCH_FINALIZE_FIXED without them otherwise); stage-out.  Every launch shape
// is fixed by `shape`, so the parts an epoch needs are captured once into one
// graph per epoch form and replayed with new table contents; timing events,
// record nodes of that graph, bracket the simulation parts.
enum {
    EPOCH_STAGE_IN = 0,
    EPOCH_SIMULATE = 1,  // + class
    EPOCH_FINALIZE = EPOCH_SIMULATE + N_CLASSES,
    EPOCH_STAGE_OUT,
    EPOCH_FINALIZE_FIXED,
    EPOCH_PARTS
};
hipError_t issue_epoch_part(int part, const EpochDevPtrs &p, const EpochShape &shape, hipStream_t s);

hipError_t launch_philox(uint64_t seed, uint64_t first, uint64_t n, uint32_t block,
                         uint32_t purpose, uint32_t *out, hipStream_t s);
hipError_t launch_normals(uint64_t seed, uint64_t first, uint64_t n, uint32_t m, float *out,
                          hipStream_t s);

}  // namespace pps
