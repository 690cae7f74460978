// Weak-informativity test (Sec. 4.1): launch descriptors shared by the HIP
// kernels in pps_smc.hip and the C-ABI entry points in pps_smc_abi.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pps.h"

namespace pps {

// Stream purposes of the test (counter word 1).
enum : uint32_t {
    SMC_P_DATA_BASE = 0x40000000u,  // D_0^(i), draw = i
    SMC_P_DATA_K = 0x40000001u,     // D_k^(i), draw = k N + i
    SMC_P_INIT = 0x50000000u,       // + particle, block 0
    SMC_P_RESAMPLE = 0x60000000u,   // + particle, block = step
    SMC_P_MCMC = 0x70000000u,       // + particle, block = 256 step + move
};
constexpr int SMC_BLOCKS_PER_STEP = 256;

// The dose-response design, passed by value to the kernels.
struct BioDesign {
    int32_t n_groups;
    int32_t n_trials[PPS_BIO_MAX_GROUPS];
    double dose[PPS_BIO_MAX_GROUPS];
};

struct SmcParams {
    int32_t n_particles;
    int32_t max_mcmc;
    int32_t max_steps;
    int32_t bisect_iters;
    double c;
    double h;
};

// The SMC runs of one launch.  mode 0: run r estimates p(y[r] | lam[r]) with
// stream index first_run + r, result in out0[r].  mode 1 (Alg. 2): run r =
// (k N + i) 2 + kind estimates p(D | lam[k]) for D = y[i] (kind 0, the base
// data sets) or yk[k N + i] (kind 1), stream index r, result in out0[k N + i]
// (kind 0) or outk[k N + i] (kind 1).  lcoef holds sum_i log C(n_i, y_i) of
// every data set (mode 0: per run; mode 1: the N base sets, then yk's).
struct SmcRuns {
    int32_t mode;
    int32_t pad;
    uint64_t n_runs;
    uint64_t n_data;
    uint64_t first_run;
    const int32_t *y;
    const int32_t *yk;
    const double *lam;
    const double *lcoef;
    double *out0;
    double *outk;
    unsigned long long *next_run;  // tile counter, zero at launch
};

// Blocks of the SMC kernel for n_particles (256, 512 or 1024 lanes).
int smc_block_for(int n_particles);
hipError_t smc_occupancy(int block, int *blocks_per_cu);

hipError_t launch_bio_data(const BioDesign &b, const double *lam, int n_lambda, uint64_t n_data,
                           uint64_t seed, int32_t *y0, int32_t *yk, double *lcoef, hipStream_t s);
hipError_t launch_smc(const BioDesign &b, const SmcParams &p, uint64_t seed, const SmcRuns &runs,
                      unsigned grid, hipStream_t s);
// p-value counts c = #{j : zk[j] <= z0[i]} per (k, i), the p-values c / N
// (when pvals != null), and gamma[k] = the q-th smallest p-value of row k.
hipError_t launch_wip_tally(const double *z0, const double *zk, int n_lambda, uint64_t n_data,
                            uint64_t q, uint32_t *counts, double *pvals, double *gamma,
                            hipStream_t s);

}  // namespace pps
