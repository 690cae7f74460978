// Internal structures shared by the host runtime and the HIP kernels of
// libpps.  Not part of the public ABI (see include/pps.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pps.h"

namespace pps {

// Job flags: what a job does with each simulated draw.
enum : int32_t {
    JOB_WRITE_DIST = 1 << 0,  // write rho_i to job.dist (ABC)
    JOB_TALLY_STAT = 1 << 1,  // count T_i >= t_obs into job.counts[0] (p-value)
    JOB_TALLY_SUMM = 1 << 2,  // count S_s(D_i) >= summ_obs[s] into job.counts[s]
    JOB_DUMP = 1 << 3,        // write theta / summaries / stat / dist per draw
    JOB_EVENTS = 1 << 4,      // tuberculosis: write events / status per draw
};

// Model classes compiled into separate simulation kernels.  CLASS_GROUP
// holds p-value rows of one lambda grid in groups of GROUP_LPL consecutive
// rows that differ only in the prior of parameter `lambda_param`: one lane
// simulates a draw under every lambda of its group from one random stream
// (common random numbers).  CLASS_CELLS runs one draw per workgroup with the
// draw's cells across the lanes (the toggle switch): a tile is one draw.
// CLASS_GILLESPIE runs one tuberculosis draw per 64-lane workgroup (its
// genotype counts in LDS): a tile is one draw, so a workgroup that finishes
// a short epidemic takes the next draw at once.
enum : int {
    CLASS_PATH = 0,
    CLASS_GARCH = 1,
    CLASS_GROUP = 2,
    CLASS_CELLS = 3,
    CLASS_GILLESPIE = 4,
    N_CLASSES = 5
};
constexpr int GROUP_LPL = 32;

// Prior parameters held by the one-lane-per-draw kernels (logistic SDE,
// normal-mean, GARCH: at most 3 used); the cell kernel holds PPS_MAX_PARAMS.
constexpr int SDE_MAX_PARAMS = 4;

// Row flags handled by the epoch stage-in / stage-out kernels.
enum : uint32_t {
    ROW_ZERO_COUNTS = 1u << 0,  // zero counts[0 .. n_counts) before simulating
    ROW_COPY_COUNTS = 1u << 1,  // copy counts[0 .. n_counts) to the host after
};

struct PriorDev {
    int32_t family;
    int32_t pad;
    double a, b;
};

// One row of the device job table.  A launch processes the tiles
// [tile_begin, tile_begin + n_tiles) of the launch's global tile range for
// this job; local tile t of the job covers draws
// [t * tile_size, (t + 1) * tile_size) of the job, clipped to n_draws.
struct alignas(16) JobDev {
    int32_t model;
    int32_t flags;
    int32_t n_params;
    int32_t n_summ;
    int32_t steps;
    int32_t obs_stride;
    int32_t constraint;
    int32_t tile_size;
    int32_t n_cells;       // CLASS_CELLS: cells per draw; CLASS_GILLESPIE: stop size
    int32_t n_sample;      // CLASS_GILLESPIE: cases sampled
    uint64_t seed;
    uint64_t first_draw;
    uint64_t n_draws;
    uint64_t tile_begin;   // first global tile id of this row in the launch
    uint64_t n_tiles;      // tiles of this row in the launch
    uint64_t tile_offset;  // first local tile of the job processed in the launch
    PriorDev prior[PPS_MAX_PARAMS];
    double x0;
    double dt;
    double noise_sd;
    double t_obs;
    double summ_obs[PPS_MAX_OBS];  // JOB_TALLY_SUMM: observed summaries (FP64)
    float y_obs[PPS_MAX_OBS];
    float *dist;                 // JOB_WRITE_DIST: n_draws floats
    unsigned long long *counts;  // tallies
    float *dump_theta;           // JOB_DUMP outputs (SoA, stride n_draws), may be null
    float *dump_summ;
    float *dump_stat;
    float *dump_dist;
    unsigned long long *dump_events;  // JOB_EVENTS (may be null)
    int32_t *dump_status;
    uint32_t row_flags;          // ROW_* above
    uint32_t n_counts;           // tallies of this row (1, or 14 for GARCH)
    uint32_t out_slot;           // ROW_COPY_COUNTS: first host slot
    int32_t lambda_param;        // CLASS_GROUP: the parameter whose prior varies
};

// Device-side launch state of one simulation class (reset by the stage-in
// kernel of each epoch).
struct alignas(64) LaunchState {
    unsigned long long next_tile;
    unsigned long long pad[7];
};

// Capacities of one epoch.
constexpr int MAX_ROWS = 4096;
constexpr int MAX_FINS = 1024;
constexpr int MAX_OUT_COUNTS = 16384;

// Epoch descriptor: staged from pinned host memory to the device at the start
// of every epoch.  Rows of class c are rows [class_first[c], class_first[c] +
// class_rows[c]) and their tiles are numbered 0 .. class_tiles[c] - 1.
struct alignas(64) EpochHeader {
    uint32_t class_first[N_CLASSES];
    uint32_t class_rows[N_CLASSES];
    uint64_t class_tiles[N_CLASSES];
    uint32_t n_rows;
    uint32_t n_fins;
    uint64_t fin_blocks;
    uint32_t any_top;
    uint32_t pad;
    uint64_t epoch_id;
};

// ---- ABC finalisation (select / compaction / moments) -------------------

// Elements per compaction / histogram workgroup: 4 waves x 32 rows x 64
// (1221 blocks at 1e7 draws: about one round of the compaction kernel's
// resident workgroups, where 16 rows took three).
constexpr int FIN_BLOCK = 256;
constexpr int FIN_ROWS = 32;
constexpr int FIN_TILE = FIN_BLOCK * FIN_ROWS;
constexpr int SEL_BITS0 = 11, SEL_BITS1 = 11, SEL_BITS2 = 10;
constexpr int SEL_BINS = 1 << 11;

struct alignas(16) FinJob {
    const float *dist;          // rho_i, n floats
    uint64_t n;
    uint64_t first_draw;
    uint64_t seed;
    int32_t mode;               // PPS_EPS_FIXED / PPS_EPS_TOP_FRACTION
    int32_t n_params;
    int32_t constraint;
    int32_t pad;
    double eps;                 // FIXED threshold
    uint64_t k;                 // TOP_FRACTION: number to accept
    uint64_t capacity;
    uint64_t block_begin;       // first global finalisation block of this job
    uint64_t n_blocks;
    PriorDev prior[PPS_MAX_PARAMS];
    uint64_t *acc_idx;
    float *acc_theta;
    float *acc_dist;
    // scratch (device, owned by the library)
    unsigned int *hist;         // SEL_BINS counters
    unsigned long long *block_counts;  // 2 * n_blocks: (lt, eq) per block, then offsets
    double *partials;           // n_blocks * (1 + 2 * n_params): (n, mean[], m2[])
    struct FinResult *result;   // device result row
};

struct alignas(16) FinResult {
    uint64_t n_accepted;
    double eps_used;
    double mean[PPS_MAX_PARAMS];
    double var[PPS_MAX_PARAMS];
    // select state
    uint32_t sel_prefix;
    uint32_t sel_mask;
    uint64_t sel_rank;          // rank (1-based) still to find among matching
    uint64_t lt_total;
    uint64_t eq_total;
    uint64_t quota;             // ties (rho == threshold) to accept
    uint32_t thresh_bits;
    uint32_t pad;
};

}  // namespace pps
