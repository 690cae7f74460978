// BEGE log-likelihood (Sec. 4.2): launch descriptor shared by the HIP kernels
// in pps_bege.hip and the C-ABI entry point in pps_bege_abi.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pps {

constexpr int BEGE_NPAR = 11;

// One batch: n_theta parameter vectors (rows of 11, device) against one
// return series r_0..r_T (device).  shape_p / shape_n hold the shapes
// p_{t-1}, n_{t-1} that meet u_t (n_theta x T each), logdens log f(u_t)
// (n_theta x T), loglik the sums (n_theta).
struct BegeBatch {
    const double *theta;
    const double *r;
    int32_t n_theta;
    int32_t T;
    int32_t n_omega;
    int32_t chunks;        // chunks of 64 steps per vector: bege_chunks(T)
    int32_t *chunk_class;  // n_theta x chunks cost classes
    int32_t *chunk_order;  // the chunks (k chunks + c) in decreasing class
    double *shape_p;
    double *shape_n;
    double *logdens;
    double *loglik;
    double *ops;  // when not null: FP64 operations of the density kernel added here
};

int bege_chunks(int T);

// Shapes, chunk order, transition densities, then the per-vector sums, in
// stream order.
// When ev0/ev1 are given they bracket the density kernel; when b.ops is set
// the density kernel is the operation-counting instantiation.
hipError_t launch_bege(const BegeBatch &b, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);

}  // namespace pps
