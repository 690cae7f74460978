// HIP kernels of the prior-predictive sampler for gfx950 (MI355X).
//
// k_simulate      persistent tile-queue kernel: one lane per prior draw;
//                 theta ~ prior (FP64, rounded to FP32), then the model
//                 simulated in VGPRs with its Philox stream regenerated in
//                 registers (no random-number buffers), then per-draw
//                 epilogues: rho to HBM (ABC), tail-area tallies by wave
//                 ballot + popcount (p-values), or a full per-draw dump.
// k_simulate_group  p-value grids: one lane simulates a draw under 8 lambda
//                 values of a grid from one random stream.
// k_simulate_cells  the toggle switch: one draw per workgroup, its cells
//                 across the lanes, their measurements sorted in LDS and
//                 reduced to quantile summaries on the CU.
// k_sel_*         radix select of the k-th smallest rho on its FP32 bit
//                 pattern (rho >= 0, so bit order = value order): 11/11/10
//                 bit digits, LDS histograms merged into a global histogram.
// k_compact_*     ordered stream compaction of accepted draws (wave ballot +
//                 mbcnt rank, LDS prefix over waves, scanned block offsets),
//                 so records come out in increasing draw index with no sort.
// k_moments_final FP64 posterior mean / variance of the accepted theta from
//                 per-block (n, mean, M2) partials combined in block order.
#include <hip/hip_runtime.h>

#include "pps_device.hpp"
#include "pps_internal.hpp"
#include "pps_launch.hpp"

namespace pps {

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// A float known to be equal in every lane, moved to a scalar register.
__device__ __forceinline__ float wave_uniform_f32(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// ===========================================================================
// Per-draw simulators.  Each returns the summaries the epilogue needs.
// ===========================================================================

// Stochastic logistic SDE by Euler-Maruyama, increment form, absorbed at 0:
//   X <- max(0, X + X (a - b X + c z)), a = th1 dt, b = th1 dt / th2,
//   c = th3 sqrt(dt).  Observation k = X after step k * stride.
// Accumulates rho^2 = sum_k (X_k - y_k)^2 and sum_k X_k with Kahan sums.
template <bool DUMP>
__device__ __forceinline__ void sim_logistic(const JobDev *__restrict__ J, StreamKey key,
                                             uint64_t draw, const double *theta, uint64_t q,
                                             bool valid, Kahan &d2, Kahan &sum)
{
    const double dt = J->dt;
    const float a = static_cast<float>(theta[0] * dt);
    const float b = static_cast<float>(theta[0] * dt / theta[1]);
    const float c = static_cast<float>(theta[2] * sqrt(dt));
    const int steps = J->steps;
    const int stride = J->obs_stride;
    const uint64_t n = J->n_draws;
    float x = static_cast<float>(J->x0);
    int next_obs = stride;
    int k = 0;
    const int nblk = (steps + NORMALS_PER_BLOCK - 1) / NORMALS_PER_BLOCK;
    for (int blk = 0; blk < nblk; ++blk) {
        float z[NORMALS_PER_BLOCK];
        path_normals6(key, draw, static_cast<uint32_t>(blk), z);
#pragma unroll
        for (int j = 0; j < NORMALS_PER_BLOCK; ++j) {
            const int step = NORMALS_PER_BLOCK * blk + j + 1;  // steps done after this update
            if (step > steps)
                break;
            float g = __builtin_fmaf(-b, x, a);
            g = __builtin_fmaf(c, z[j], g);
            x = __builtin_fmaxf(__builtin_fmaf(x, g, x), 0.0f);
            if (step == next_obs) {
                const float diff = x - J->y_obs[k];
                d2.add(diff * diff);
                sum.add(x);
                if (DUMP && valid && J->dump_summ)
                    J->dump_summ[static_cast<uint64_t>(k) * n + q] = x;
                ++k;
                next_obs += stride;
            }
        }
    }
}

// Normal-mean model: y_j = mu + sd z_j.
template <bool DUMP>
__device__ __forceinline__ void sim_normal_mean(const JobDev *__restrict__ J, StreamKey key,
                                                uint64_t draw, const double *theta, uint64_t q,
                                                bool valid, Kahan &d2, Kahan &sum)
{
    const float mu = static_cast<float>(theta[0]);
    const float sd = static_cast<float>(J->noise_sd);
    const int m = J->n_summ;
    const uint64_t n = J->n_draws;
    const int nblk = (m + NORMALS_PER_BLOCK - 1) / NORMALS_PER_BLOCK;
    for (int blk = 0; blk < nblk; ++blk) {
        float z[NORMALS_PER_BLOCK];
        path_normals6(key, draw, static_cast<uint32_t>(blk), z);
#pragma unroll
        for (int j = 0; j < NORMALS_PER_BLOCK; ++j) {
            const int k = NORMALS_PER_BLOCK * blk + j;
            if (k >= m)
                break;
            const float y = __builtin_fmaf(sd, z[j], mu);
            const float diff = y - J->y_obs[k];
            d2.add(diff * diff);
            sum.add(y);
            if (DUMP && valid && J->dump_summ)
                J->dump_summ[static_cast<uint64_t>(k) * n + q] = y;
        }
    }
}

// GARCH(1,1) in scaled form.  With sbar^2 = omega/(1-alpha-beta),
// s_t = r_t / sbar and h_t = sigma2_t / sbar^2, the recursion
// sigma2_{t+1} = omega + alpha r_t^2 + beta sigma2_t becomes, exactly,
//   h_1 = 1,  s_t = sqrt(h_t) z_t,  h_{t+1} = (1-alpha-beta) + alpha s_t^2 + beta h_t.
// The variance ratio h is carried in FP64 with alpha, beta and 1-alpha-beta
// unrounded: with persistence alpha+beta near 1 the recursion keeps an error
// in its state for ~1/(1-alpha-beta) steps, so an FP32 state (or FP32
// alpha, beta) moves the variance and kurtosis of near-integrated draws by
// up to ~1e-4.  Normals, returns s_t and every summary stay FP32; the state
// costs two FP64 FMAs and two conversions per step.
// Streaming summaries: plain FP32 sums over 20-step blocks folded into Kahan
// totals; b_t = s_t^2 - 1 kept in a 10-deep register ring for the lag
// products; the first 10 b_t are recomputed from the stream at the end for
// the ACF centring terms.  The closing algebra is FP64.  Requires the length
// to be a multiple of 20; the steps run in spans of 60 (ten blocks of six
// normals, three folds), the last span possibly cut to 20 or 40.
__device__ __forceinline__ float garch_step(double &h, float z, double al, double be, double c)
{
    const float s = __builtin_amdgcn_sqrtf(static_cast<float>(h)) * z;
    const float sq = s * s;
    h = __builtin_fma(al, static_cast<double>(sq), __builtin_fma(be, h, c));
    return s;
}

__device__ __forceinline__ void sim_garch(const JobDev *__restrict__ J, StreamKey key,
                                          uint64_t draw, const double *theta, double *summ)
{
    const double alpha_d = theta[1], beta_d = theta[2];
    const double oab = 1.0 - alpha_d - beta_d;
    const int len = J->steps;
    double h = 1.0;
    Kahan K1, K2, K3, K4, KL[PPS_GARCH_LAGS];
    float ring[PPS_GARCH_LAGS];
#pragma unroll
    for (int k = 0; k < PPS_GARCH_LAGS; ++k)
        ring[k] = 0.0f;
    float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
    float lag[PPS_GARCH_LAGS];
#pragma unroll
    for (int k = 0; k < PPS_GARCH_LAGS; ++k)
        lag[k] = 0.0f;
    // The step at position jj of its 60-step span (10 Philox blocks; spans
    // start at multiples of 60, so jj % 10 is the step's ring slot); every
    // 20th step folds the block sums into the Kahan totals.
    auto step = [&](int jj, float zj) {
        const float s = garch_step(h, zj, alpha_d, beta_d, oab);
        const float sq = s * s;
        s1 += s;
        s2 += sq;
        s3 = __builtin_fmaf(sq, s, s3);
        s4 = __builtin_fmaf(sq, sq, s4);
        const float bt = sq - 1.0f;
#pragma unroll
        for (int k = 1; k <= PPS_GARCH_LAGS; ++k)
            lag[k - 1] = __builtin_fmaf(bt, ring[(jj - k + 60) % 10], lag[k - 1]);
        ring[jj % 10] = bt;
        if (jj % 20 == 19) {
            K1.add(s1);
            K2.add(s2);
            K3.add(s3);
            K4.add(s4);
            s1 = s2 = s3 = s4 = 0.0f;
#pragma unroll
            for (int k = 0; k < PPS_GARCH_LAGS; ++k) {
                KL[k].add(lag[k]);
                lag[k] = 0.0f;
            }
        }
    };
    // The first `lim` steps of span sp (lim = 60 but in the last span).
    auto span = [&](int sp, int lim) {
#pragma unroll
        for (int p = 0; p < 10; ++p) {
            if (NORMALS_PER_BLOCK * p >= lim)
                break;
            float z[NORMALS_PER_BLOCK];
            path_normals6<false>(key, draw, static_cast<uint32_t>(10 * sp + p), z);
#pragma unroll
            for (int j = 0; j < NORMALS_PER_BLOCK; ++j)
                if (NORMALS_PER_BLOCK * p + j < lim)
                    step(NORMALS_PER_BLOCK * p + j, z[j]);
        }
    };
    const int nspan = len / 60;
    for (int sp = 0; sp < nspan; ++sp)
        span(sp, 60);
    if (len > 60 * nspan)
        span(nspan, len - 60 * nspan);  // 20 or 40 steps
    // The first 10 b_t again (same operations, so the same values).
    float head[PPS_GARCH_LAGS];
    {
        double h0 = 1.0;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float z[NORMALS_PER_BLOCK];
            path_normals6<false>(key, draw, static_cast<uint32_t>(p), z);
#pragma unroll
            for (int j = 0; j < NORMALS_PER_BLOCK; ++j) {
                if (NORMALS_PER_BLOCK * p + j < PPS_GARCH_LAGS) {
                    const float s = garch_step(h0, z[j], alpha_d, beta_d, oab);
                    head[NORMALS_PER_BLOCK * p + j] = s * s - 1.0f;
                }
            }
        }
    }
    // Closing algebra in FP64.
    const double T = static_cast<double>(len);
    const double S1 = K1.value(), S2 = K2.value(), S3 = K3.value(), S4 = K4.value();
    const double m = S1 / T, e2 = S2 / T, e3 = S3 / T, e4 = S4 / T;
    const double m2 = e2 - m * m;
    const double m3 = e3 - 3.0 * m * e2 + 2.0 * m * m * m;
    const double m4 = e4 - 4.0 * m * e3 + 6.0 * m * m * e2 - 3.0 * m * m * m * m;
    const double sbar2 = theta[0] / oab;
    summ[0] = sqrt(sbar2) * m;
    summ[1] = sbar2 * m2;
    summ[2] = m3 / (m2 * sqrt(m2));
    summ[3] = m4 / (m2 * m2);
    // ACF of r^2: a_t - abar = sbar^2 (b_t - bbar), bbar = S2/T - 1.
    const double B = S2 - T;
    const double bbar = B / T;
    const double den = (S4 - 2.0 * S2 + T) - T * bbar * bbar;
    // tail_k = sum of the last k b_t: b_{len-m} sits in ring[(len-m) % 10],
    // and len is a multiple of 20, so b_{len-m} = ring[(20-m) % 10].
    double headk = 0.0, tailk = 0.0;
#pragma unroll
    for (int k = 1; k <= PPS_GARCH_LAGS; ++k) {
        headk += static_cast<double>(head[k - 1]);
        tailk += static_cast<double>(ring[(20 - k) % 10]);
        const double num = KL[k - 1].value() - bbar * ((B - tailk) + (B - headk)) +
                           (T - k) * bbar * bbar;
        summ[3 + k] = num / den;
    }
}

// The same logistic simulation for DPL independent draws per lane, with
// UNROLL Philox blocks generated per loop trip: the draws' (and blocks')
// random streams are independent, which gives the scheduler instruction-level
// parallelism without changing any draw's arithmetic.
template <int DPL, int UNROLL>
__device__ __forceinline__ void sim_logistic_ilp(const JobDev *__restrict__ J, StreamKey key,
                                                 const uint64_t (&draw)[DPL],
                                                 const double (&theta)[DPL][SDE_MAX_PARAMS],
                                                 Kahan (&d2)[DPL], Kahan (&sum)[DPL])
{
    const double dt = J->dt;
    const double sdt = sqrt(dt);
    float a[DPL], b[DPL], c[DPL], x[DPL];
#pragma unroll
    for (int d = 0; d < DPL; ++d) {
        a[d] = static_cast<float>(theta[d][0] * dt);
        b[d] = static_cast<float>(theta[d][0] * dt / theta[d][1]);
        c[d] = static_cast<float>(theta[d][2] * sdt);
        x[d] = static_cast<float>(J->x0);
    }
    const int steps = J->steps;
    const int stride = J->obs_stride;
    const int nblk = (steps + NORMALS_PER_BLOCK - 1) / NORMALS_PER_BLOCK;
    int next_obs = stride;
    int k = 0;
    int blk = 0;
    for (; blk + UNROLL <= nblk; blk += UNROLL) {
        float z[UNROLL][DPL][NORMALS_PER_BLOCK];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int d = 0; d < DPL; ++d)
                path_normals6(key, draw[d], static_cast<uint32_t>(blk + u), z[u][d]);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
            for (int j = 0; j < NORMALS_PER_BLOCK; ++j) {
                const int step = NORMALS_PER_BLOCK * (blk + u) + j + 1;
                if (step > steps)
                    break;
#pragma unroll
                for (int d = 0; d < DPL; ++d) {
                    float g = __builtin_fmaf(-b[d], x[d], a[d]);
                    g = __builtin_fmaf(c[d], z[u][d][j], g);
                    x[d] = __builtin_fmaxf(__builtin_fmaf(x[d], g, x[d]), 0.0f);
                }
                if (step == next_obs) {
                    const float y = J->y_obs[k];
#pragma unroll
                    for (int d = 0; d < DPL; ++d) {
                        const float diff = x[d] - y;
                        d2[d].add(diff * diff);
                        sum[d].add(x[d]);
                    }
                    ++k;
                    next_obs += stride;
                }
            }
        }
    }
    for (; blk < nblk; ++blk) {
        float z[DPL][NORMALS_PER_BLOCK];
#pragma unroll
        for (int d = 0; d < DPL; ++d)
            path_normals6(key, draw[d], static_cast<uint32_t>(blk), z[d]);
#pragma unroll
        for (int j = 0; j < NORMALS_PER_BLOCK; ++j) {
            const int step = NORMALS_PER_BLOCK * blk + j + 1;
            if (step > steps)
                break;
#pragma unroll
            for (int d = 0; d < DPL; ++d) {
                float g = __builtin_fmaf(-b[d], x[d], a[d]);
                g = __builtin_fmaf(c[d], z[d][j], g);
                x[d] = __builtin_fmaxf(__builtin_fmaf(x[d], g, x[d]), 0.0f);
            }
            if (step == next_obs) {
                const float y = J->y_obs[k];
#pragma unroll
                for (int d = 0; d < DPL; ++d) {
                    const float diff = x[d] - y;
                    d2[d].add(diff * diff);
                    sum[d].add(x[d]);
                }
                ++k;
                next_obs += stride;
            }
        }
    }
}

// ===========================================================================
// Persistent simulation kernel.
//
// CLASS selects the model family compiled into this instance, so that each
// family gets its own register allocation: CLASS_PATH = logistic SDE and
// normal-mean (short per-draw state), CLASS_GARCH = GARCH(1,1) (summary ring).
// A tile is BLOCK * DPL draws of one job row; lane t handles draws
// q0 + t + d * BLOCK, d < DPL.  Workgroups pull tiles from an atomic counter
// until the class's tiles of the epoch are exhausted.
// ===========================================================================
template <int BLOCK, int CLASS, int DPL, int UNROLL>
__global__ __launch_bounds__(BLOCK) void k_simulate(const EpochHeader *__restrict__ hdr,
                                                    const JobDev *__restrict__ rows,
                                                    LaunchState *__restrict__ states)
{
    constexpr int NW = BLOCK / 64;
    __shared__ unsigned long long s_tile;
    __shared__ unsigned s_cnt[PPS_GARCH_NSUMM][NW];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int n_jobs = static_cast<int>(hdr->class_rows[CLASS]);
    const uint64_t total_tiles = hdr->class_tiles[CLASS];
    const JobDev *__restrict__ jobs = rows + hdr->class_first[CLASS];
    LaunchState *__restrict__ state = states + CLASS;
    for (;;) {
        if (tid == 0)
            s_tile = atomicAdd(&state->next_tile, 1ull);
        __syncthreads();
        const uint64_t t = uniform_u64(s_tile);
        __syncthreads();
        if (t >= total_tiles)
            break;
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const JobDev *__restrict__ J = jobs + lo;
        const int flags = J->flags;
        const uint64_t n = J->n_draws;
        const uint64_t q0 = (t - J->tile_begin + J->tile_offset) * static_cast<uint64_t>(J->tile_size);
        const StreamKey key = make_key(J->seed);
        const bool wave_live = q0 + static_cast<uint64_t>(wave) * 64 < n;
        uint64_t q[DPL], draw[DPL];
        bool valid[DPL];
#pragma unroll
        for (int d = 0; d < DPL; ++d) {
            q[d] = q0 + static_cast<uint64_t>(tid + d * BLOCK);
            valid[d] = q[d] < n;
            draw[d] = J->first_draw + q[d];
        }
        double theta[DPL][SDE_MAX_PARAMS];
        double summ[PPS_GARCH_NSUMM];
        Kahan d2[DPL], sum[DPL];
#pragma unroll
        for (int d = 0; d < DPL; ++d)
#pragma unroll
            for (int j = 0; j < SDE_MAX_PARAMS; ++j)
                theta[d][j] = 0.0;
        const int model = J->model;
        if (wave_live) {
#pragma unroll
            for (int d = 0; d < DPL; ++d)
                prior_draw<SDE_MAX_PARAMS>(J->prior, J->n_params, J->constraint, key, draw[d], theta[d]);
            if constexpr (CLASS == CLASS_GARCH) {
                sim_garch(J, key, draw[0], theta[0], summ);
            } else {
                if (model == PPS_LOGISTIC_SDE && !(flags & JOB_DUMP)) {
                    sim_logistic_ilp<DPL, UNROLL>(J, key, draw, theta, d2, sum);
                } else {
#pragma unroll
                    for (int d = 0; d < DPL; ++d) {
                        if (model == PPS_LOGISTIC_SDE)
                            sim_logistic<true>(J, key, draw[d], theta[d], q[d], valid[d], d2[d], sum[d]);
                        else if (flags & JOB_DUMP)
                            sim_normal_mean<true>(J, key, draw[d], theta[d], q[d], valid[d], d2[d], sum[d]);
                        else
                            sim_normal_mean<false>(J, key, draw[d], theta[d], q[d], valid[d], d2[d], sum[d]);
                    }
                }
            }
        }
        constexpr bool garch = CLASS == CLASS_GARCH;
        float dist[DPL];
        double stat[DPL];
#pragma unroll
        for (int d = 0; d < DPL; ++d) {
            dist[d] = garch ? 0.0f : static_cast<float>(sqrt(d2[d].value()));
            stat[d] = garch ? 0.0 : sum[d].value() / static_cast<double>(J->n_summ);
        }
#pragma unroll
        for (int d = 0; d < DPL; ++d) {
            if ((flags & JOB_WRITE_DIST) && valid[d])
                J->dist[q[d]] = dist[d];
            if ((flags & JOB_DUMP) && valid[d]) {
                if (J->dump_theta)
                    for (int j = 0; j < J->n_params; ++j)
                        J->dump_theta[static_cast<uint64_t>(j) * n + q[d]] = static_cast<float>(theta[d][j]);
                if (garch && J->dump_summ)
                    for (int s = 0; s < PPS_GARCH_NSUMM; ++s)
                        J->dump_summ[static_cast<uint64_t>(s) * n + q[d]] = static_cast<float>(summ[s]);
                if (!garch && J->dump_stat)
                    J->dump_stat[q[d]] = static_cast<float>(stat[d]);
                if (!garch && J->dump_dist)
                    J->dump_dist[q[d]] = dist[d];
            }
        }
        if (flags & (JOB_TALLY_STAT | JOB_TALLY_SUMM)) {
            const int ns = (flags & JOB_TALLY_SUMM) ? (garch ? PPS_GARCH_NSUMM : 0) : 1;
            for (int s = 0; s < ns; ++s) {
                unsigned cnt = 0;
#pragma unroll
                for (int d = 0; d < DPL; ++d) {
                    const double v = (flags & JOB_TALLY_SUMM) ? summ[s] : stat[d];
                    const double ref = (flags & JOB_TALLY_SUMM) ? J->summ_obs[s] : J->t_obs;
                    cnt += static_cast<unsigned>(__popcll(__ballot(valid[d] && v >= ref)));
                }
                if (lane_id() == 0)
                    s_cnt[s][wave] = cnt;
            }
            __syncthreads();
            if (tid < ns) {
                unsigned tot = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    tot += s_cnt[tid][w];
                if (tot)
                    atomicAdd(&J->counts[tid], static_cast<unsigned long long>(tot));
            }
        }
    }
}

// ===========================================================================
// Lambda-group kernel (p-value grids, logistic SDE).  One lane simulates draw
// i under the LPL lambda values of its group: the path normals and every
// prior parameter except `lambda_param` are shared (common random numbers),
// and so is the variate of `lambda_param` itself, to which each member
// applies its own prior; each member keeps its own state, the EM constants
// that depend on the varied parameter, and its compensated mean, and tallies
// its own statistic.  The member arithmetic is the same sequence of
// operations as in k_simulate, so counts equal those of one row per lambda.
// ===========================================================================

// The members' Euler-Maruyama runs of one draw; VARY is the varied
// parameter (0: a and b depend on it, 1: b, 2: c), the other constants are
// held once.
template <int LPL, int VARY>
__device__ __forceinline__ void group_members(const JobDev *__restrict__ J, StreamKey key,
                                              uint64_t draw, const double *theta, double u,
                                              double zv, Kahan *sum)
{
    constexpr int NA = VARY == 0 ? LPL : 1;
    constexpr int NB = VARY <= 1 ? LPL : 1;
    constexpr int NC = VARY == 2 ? LPL : 1;
    const double dt = J->dt;
    const double sdt = sqrt(dt);
    float a[NA], b[NB], c[NC], x[LPL];
#pragma unroll
    for (int k = 0; k < LPL; ++k) {
        double th[3] = {theta[0], theta[1], theta[2]};
        th[VARY] = prior_transform(J[k].prior[VARY], u, zv);
        if (k < NA)
            a[k] = static_cast<float>(th[0] * dt);
        if (k < NB)
            b[k] = static_cast<float>(th[0] * dt / th[1]);
        if (k < NC)
            c[k] = static_cast<float>(th[2] * sdt);
        x[k] = static_cast<float>(J->x0);
    }
    const int steps = J->steps;
    const int stride = J->obs_stride;
    const int nblk = (steps + NORMALS_PER_BLOCK - 1) / NORMALS_PER_BLOCK;
    int next_obs = stride;
    // the normals of block blk + 1 are generated while the members advance
    // through block blk: the two are independent, so the scheduler can fill
    // the Philox / Box-Muller latencies with member updates
    float zn[NORMALS_PER_BLOCK];
    path_normals6(key, draw, 0u, zn);
    for (int blk = 0; blk < nblk; ++blk) {
        float z[NORMALS_PER_BLOCK];
#pragma unroll
        for (int j = 0; j < NORMALS_PER_BLOCK; ++j)
            z[j] = zn[j];
        if (blk + 1 < nblk)
            path_normals6(key, draw, static_cast<uint32_t>(blk + 1), zn);
#pragma unroll
        for (int j = 0; j < NORMALS_PER_BLOCK; ++j) {
            const int step = NORMALS_PER_BLOCK * blk + j + 1;
            if (step > steps)
                break;
#pragma unroll
            for (int k = 0; k < LPL; ++k) {
                float g = __builtin_fmaf(-b[k < NB ? k : 0], x[k], a[k < NA ? k : 0]);
                g = __builtin_fmaf(c[k < NC ? k : 0], z[j], g);
                x[k] = __builtin_fmaxf(__builtin_fmaf(x[k], g, x[k]), 0.0f);
            }
            if (step == next_obs) {
#pragma unroll
                for (int k = 0; k < LPL; ++k)
                    sum[k].add(x[k]);
                next_obs += stride;
            }
        }
    }
}

template <int BLOCK, int LPL>
__global__ __launch_bounds__(BLOCK) void k_simulate_group(const EpochHeader *__restrict__ hdr,
                                                          const JobDev *__restrict__ rows,
                                                          LaunchState *__restrict__ states)
{
    constexpr int NW = BLOCK / 64;
    __shared__ unsigned long long s_tile;
    __shared__ unsigned s_cnt[LPL][NW];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int n_groups = static_cast<int>(hdr->class_rows[CLASS_GROUP] / LPL);
    const uint64_t total_tiles = hdr->class_tiles[CLASS_GROUP];
    const JobDev *__restrict__ grp = rows + hdr->class_first[CLASS_GROUP];
    LaunchState *__restrict__ state = states + CLASS_GROUP;
    for (;;) {
        if (tid == 0)
            s_tile = atomicAdd(&state->next_tile, 1ull);
        __syncthreads();
        const uint64_t t = uniform_u64(s_tile);
        __syncthreads();
        if (t >= total_tiles)
            break;
        int lo = 0, hi = n_groups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (grp[mid * LPL].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const JobDev *__restrict__ J = grp + lo * LPL;
        const uint64_t n = J->n_draws;
        const uint64_t q0 = (t - J->tile_begin + J->tile_offset) * static_cast<uint64_t>(J->tile_size);
        const uint64_t q = q0 + static_cast<uint64_t>(tid);
        const bool valid = q < n;
        const bool wave_live = q0 + static_cast<uint64_t>(wave) * 64 < n;
        const uint64_t draw = J->first_draw + q;
        const StreamKey key = make_key(J->seed);
        Kahan sum[LPL];
        if (wave_live) {
            double theta[SDE_MAX_PARAMS] = {0.0, 0.0, 0.0, 0.0};
            prior_draw<SDE_MAX_PARAMS>(J->prior, J->n_params, J->constraint, key, draw, theta);
            const int lp = J->lambda_param;
            double u = 0.0, zv = 0.0;
            prior_variates(key, draw, lp, u, zv);
            if (lp == 0)
                group_members<LPL, 0>(J, key, draw, theta, u, zv, sum);
            else if (lp == 1)
                group_members<LPL, 1>(J, key, draw, theta, u, zv, sum);
            else
                group_members<LPL, 2>(J, key, draw, theta, u, zv, sum);
        }
        const double inv = 1.0 / static_cast<double>(J->n_summ);
#pragma unroll
        for (int k = 0; k < LPL; ++k) {
            const bool hit = valid && sum[k].value() * inv >= J[k].t_obs;
            const uint64_t m = __ballot(hit);
            if (lane_id() == 0)
                s_cnt[k][wave] = static_cast<unsigned>(__popcll(m));
        }
        __syncthreads();
        if (tid < LPL) {
            unsigned tot = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w)
                tot += s_cnt[tid][w];
            if (tot)
                atomicAdd(&J[tid].counts[0], static_cast<unsigned long long>(tot));
        }
    }
}

// ===========================================================================
// Genetic toggle switch (one draw per workgroup).
//
// A tile is one draw.  Every lane draws the same theta (FP64, rounded to
// FP32 constants), then the workgroup's lanes take the draw's cells in turn,
// each cell's two gene levels held in VGPRs for all steps with its normals
// regenerated from the cell's own stream.  The cells' measurements land in
// LDS, a bitonic sort orders them there, and the quantile summaries are read
// at their ranks: the measurements of a draw never leave the CU.
// ===========================================================================
struct ToggleConsts {
    float mu;        // mu
    float mu_sigma;  // mu * sigma
    float gamma;
    float dt_alpha_u, dt_alpha_v;  // dt alpha_u, dt alpha_v
    float beta_u, beta_v;
    float dt;        // dt
    float decay;     // 0.03 dt
    float noise;     // 0.5 sqrt(dt)
};

// One Euler-Maruyama step of one cell (Eq. gene_uv_SDE_EM) from the levels
// before the step; v^beta_u = exp2(beta_u log2 v) with the hardware log2 /
// exp2 (levels are >= 1, so log2 >= 0), the Hill factor 1 / (1 + p) by the
// hardware reciprocal.
__device__ __forceinline__ void toggle_step(const ToggleConsts &P, float &u, float &v, float xi_u,
                                            float xi_v)
{
    const float pu = __builtin_amdgcn_exp2f(P.beta_u * __builtin_amdgcn_logf(v));
    const float pv = __builtin_amdgcn_exp2f(P.beta_v * __builtin_amdgcn_logf(u));
    float du = __builtin_fmaf(-P.decay, u, -P.dt);  // -dt (1 + 0.03 u)
    float dv = __builtin_fmaf(-P.decay, v, -P.dt);
    du = __builtin_fmaf(P.dt_alpha_u, __builtin_amdgcn_rcpf(1.0f + pu), du);
    dv = __builtin_fmaf(P.dt_alpha_v, __builtin_amdgcn_rcpf(1.0f + pv), dv);
    u = __builtin_fmaxf(__builtin_fmaf(P.noise, xi_u, u + du), 1.0f);
    v = __builtin_fmaxf(__builtin_fmaf(P.noise, xi_v, v + dv), 1.0f);
}

// Measurement of one cell after `steps` steps (Eq. gene_u_obs), held at >= 1.
// Step j uses normals 2j, 2j+1 of the cell's stream (Philox block b holds
// steps 3b, 3b+1 and 3b+2); the measurement noise is normal 2 steps.
__device__ __forceinline__ float toggle_cell(const ToggleConsts &P, StreamKey key, uint64_t draw,
                                             uint32_t cell, int steps, float x0)
{
    constexpr int SPB = NORMALS_PER_BLOCK / 2;  // steps per block
    float u = x0, v = x0;
    const int full = steps / SPB;
    for (int b = 0; b < full; ++b) {
        float z[NORMALS_PER_BLOCK];
        cell_normals6(key, draw, cell, static_cast<uint32_t>(b), z);
#pragma unroll
        for (int j = 0; j < SPB; ++j)
            toggle_step(P, u, v, z[2 * j], z[2 * j + 1]);
    }
    // the last block: the remaining steps (fewer than three), then eta
    const int rest = steps - SPB * full;
    float z[NORMALS_PER_BLOCK];
    cell_normals6(key, draw, cell, static_cast<uint32_t>(full), z);
    if (rest > 0)
        toggle_step(P, u, v, z[0], z[1]);
    if (rest > 1)
        toggle_step(P, u, v, z[2], z[3]);
    const float eta = rest == 0 ? z[0] : (rest == 1 ? z[2] : z[4]);
    // u^-gamma = exp2(-gamma log2 u)
    const float scale = __builtin_amdgcn_exp2f(-P.gamma * __builtin_amdgcn_logf(u));
    const float y = __builtin_fmaf(P.mu_sigma * eta, scale, u + P.mu);
    return __builtin_fmaxf(y, 1.0f);
}

// Ascending bitonic sort of s[0 .. n2) (n2 a power of two) by the workgroup.
template <int BLOCK>
__device__ __forceinline__ void lds_bitonic_sort(float *s, unsigned n2)
{
    for (unsigned k = 2; k <= n2; k <<= 1) {
        for (unsigned j = k >> 1; j > 0; j >>= 1) {
            for (unsigned i = threadIdx.x; i < (n2 >> 1); i += BLOCK) {
                const unsigned lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const unsigned hi = lo | j;
                const float a = s[lo];
                const float b = s[hi];
                if ((a > b) == ((lo & k) == 0)) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_simulate_cells(const EpochHeader *__restrict__ hdr,
                                                          const JobDev *__restrict__ rows,
                                                          LaunchState *__restrict__ states)
{
    __shared__ unsigned long long s_tile;
    __shared__ double s_theta[PPS_MAX_PARAMS];
    __shared__ float s_q[PPS_MAX_OBS];
    __shared__ float s_y[PPS_TSW_MAX_CELLS];
    const unsigned tid = threadIdx.x;
    const int n_jobs = static_cast<int>(hdr->class_rows[CLASS_CELLS]);
    const uint64_t total_tiles = hdr->class_tiles[CLASS_CELLS];
    const JobDev *__restrict__ jobs = rows + hdr->class_first[CLASS_CELLS];
    LaunchState *__restrict__ state = states + CLASS_CELLS;
    for (;;) {
        if (tid == 0)
            s_tile = atomicAdd(&state->next_tile, 1ull);
        __syncthreads();
        const uint64_t t = uniform_u64(s_tile);
        __syncthreads();
        if (t >= total_tiles)
            break;
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const JobDev *__restrict__ J = jobs + lo;
        const int flags = J->flags;
        const uint64_t n = J->n_draws;
        const uint64_t q = t - J->tile_begin + J->tile_offset;  // one draw per tile
        const uint64_t draw = J->first_draw + q;
        const StreamKey key = make_key(J->seed);
        // theta ~ prior: lane j draws parameter j (the model has no
        // constraint, so the parameters are independent draws, attempt 0)
        if (tid < static_cast<unsigned>(J->n_params))
            s_theta[tid] = prior_value(J->prior[tid], key, draw, static_cast<int>(tid), 0);
        __syncthreads();
        ToggleConsts P;
        {
            // the same in every lane: the constants live in SGPRs
            const double dt = J->dt;
            P.mu = wave_uniform_f32(static_cast<float>(s_theta[0]));
            P.mu_sigma = wave_uniform_f32(static_cast<float>(s_theta[0] * s_theta[1]));
            P.gamma = wave_uniform_f32(static_cast<float>(s_theta[2]));
            P.dt_alpha_u = wave_uniform_f32(static_cast<float>(dt * s_theta[3]));
            P.dt_alpha_v = wave_uniform_f32(static_cast<float>(dt * s_theta[4]));
            P.beta_u = wave_uniform_f32(static_cast<float>(s_theta[5]));
            P.beta_v = wave_uniform_f32(static_cast<float>(s_theta[6]));
            P.dt = wave_uniform_f32(static_cast<float>(dt));
            P.decay = wave_uniform_f32(static_cast<float>(0.03 * dt));
            P.noise = wave_uniform_f32(static_cast<float>(0.5 * sqrt(dt)));
        }
        const unsigned n_cells = static_cast<unsigned>(J->n_cells);
        const int steps = J->steps;
        const float x0 = static_cast<float>(J->x0);
        for (unsigned c = tid; c < n_cells; c += BLOCK)
            s_y[c] = toggle_cell(P, key, draw, c, steps, x0);
        unsigned n2 = 1;
        while (n2 < n_cells)
            n2 <<= 1;
        for (unsigned c = n_cells + tid; c < n2; c += BLOCK)
            s_y[c] = __builtin_inff();
        __syncthreads();
        lds_bitonic_sort<BLOCK>(s_y, n2);
        // quantile k (1-based) is the ceil(k C / (K + 1))-th smallest value
        const int ns = J->n_summ;
        const unsigned kq = tid + 1;
        const float qv = static_cast<int>(tid) < ns
                             ? s_y[(kq * n_cells + static_cast<unsigned>(ns)) / (ns + 1) - 1]
                             : 0.0f;
        if ((flags & JOB_DUMP) && J->dump_summ && static_cast<int>(tid) < ns)
            J->dump_summ[static_cast<uint64_t>(tid) * n + q] = qv;
        if ((flags & JOB_TALLY_SUMM) && static_cast<int>(tid) < ns &&
            static_cast<double>(qv) >= J->summ_obs[tid])
            atomicAdd(&J->counts[tid], 1ull);
        if (static_cast<int>(tid) < ns)
            s_q[tid] = qv;
        if ((flags & JOB_DUMP) && J->dump_theta && static_cast<int>(tid) < J->n_params)
            J->dump_theta[static_cast<uint64_t>(tid) * n + q] = static_cast<float>(s_theta[tid]);
        __syncthreads();
        // Distance and statistic: every lane runs the same loop over the
        // quantiles in LDS (uniform control flow: no divergent loop may sit
        // between the last barrier of a tile and the first of the next).
        Kahan d2, sum;
        for (int k = 0; k < ns; ++k) {
            const float v = s_q[k];
            const float diff = v - J->y_obs[k];
            d2.add(diff * diff);
            sum.add(v);
        }
        const float dist = static_cast<float>(sqrt(d2.value()));
        const double stat = sum.value() / static_cast<double>(ns);
        if (tid == 0) {
            if (flags & JOB_WRITE_DIST)
                J->dist[q] = dist;
            if ((flags & JOB_DUMP) && J->dump_stat)
                J->dump_stat[q] = static_cast<float>(stat);
            if ((flags & JOB_DUMP) && J->dump_dist)
                J->dump_dist[q] = dist;
            if ((flags & JOB_TALLY_STAT) && stat >= J->t_obs)
                atomicAdd(&J->counts[0], 1ull);
        }
        __syncthreads();
    }
}

// ===========================================================================
// Tuberculosis transmission (App. B): one draw per 64-lane workgroup.
//
// A Gillespie run is a sequential Markov chain, so the lanes of a wave share
// one run.  The genotype slots (PPS_TB_MAX_POP of them) are cut into rows of
// 64; LDS holds each row as the inclusive prefix sums of its slots' counts
// (uint16), and registers hold, four rows per lane, the lane's cumulative
// case counts through each row and the rows' occupied-slot counts, plus each
// lane's exclusive prefix of the case counts over the lanes before it.  The
// case chosen by an event is found by a 64-way descent: a ballot over the
// lane prefixes picks the lane, the lane's compares of its cumulative counts
// the row, and a ballot over the row's prefixes the slot -- the same slot as
// the paper's linear scan over the genotype weights.  An update adds +-1 to
// the row's prefixes from the slot on (one LDS row read-modify-write) and to
// the register counts.  The lowest empty slot for a new genotype is found the
// same way from the occupied counts.  The event words of 64 Philox blocks
// (128 events) are drawn at once, one block per lane, and read out by lane
// index.  Runs end when the population reaches the stop size, dies out or
// hits the event cap, and the workgroup takes the next draw from the tile
// queue at once, so runs of very different lengths balance across the
// machine; the queue is walked twice, the runs predicted from theta to be
// long first.  The workgroup is one wave: its LDS operations complete in
// order, and wave barriers keep the compiler from reordering them.
// ===========================================================================
constexpr int TB_BLOCK = 64;
constexpr int TB_SLOTS = PPS_TB_MAX_POP;
constexpr int TB_NROW = TB_SLOTS / 64;
static_assert(TB_NROW == 4 * TB_BLOCK, "four rows per lane");
enum : int32_t { TB_COMPLETE = 0, TB_EXTINCT = 1, TB_TRUNCATED = 2 };
// bit 6 of every 16-bit field: set exactly when a row's occupied count is 64
constexpr uint64_t TB_FULL_BITS = 0x0040004000400040ull;

__device__ __forceinline__ uint64_t tb_readlane64(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), lane);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Lowest set lane of a ballot (63 for an empty one: only keeps indices in
// range; the ballots below are never empty with consistent counts).
__device__ __forceinline__ int tb_first(unsigned long long mask)
{
    return __builtin_ctzll(mask | (1ull << 63));
}

// Register half of the counts: rows 4 lane + j, j = 0..3, in 16-bit fields.
struct TbRegs {
    uint64_t cum4;  // cases in the lane's rows up to and including row j
    uint64_t occ4;  // occupied slots per row (rows past the population: 64)
    int excl;       // cases in the rows of lower lanes
};

// Two 16-bit lanes of a 32-bit register: a - b in each (v_pk_sub_u16).
typedef unsigned short tb_u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t tb_sub16x2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(tb_u16x2, a) - __builtin_bit_cast(tb_u16x2, b));
}

struct TbHit {
    int grp;         // lane holding the row's totals
    int fld;         // the row's field in that lane
    int row;         // 4 grp + fld
    int col;         // slot within the row
    int pre;         // this lane's prefix in the row
    bool from_col;   // this lane's slot is col or after it
    bool after_grp;  // this lane is after grp
};

// The slot holding case m (0 <= m < number of cases) in slot order.  Every
// lane works out, from its own cumulative row counts, which of its rows would
// hold case m and its rank there (VALU work beside the ballot that picks the
// lane); one lane read then takes the picked lane's (row, rank).
__device__ __forceinline__ TbHit tb_find(const uint16_t *pre, const TbRegs &c, uint32_t m)
{
    const int lane = threadIdx.x;
    TbHit h;
    const int r = static_cast<int>(m) - c.excl;
    // C_j - r - 1 in each 16-bit field: negative (bit 15 of the field set)
    // exactly when the lane's first j + 1 rows hold at most r cases.  In the
    // lane that holds case m, 0 <= r < C_3 <= 2^14, so every difference
    // fits in 16 signed bits (other lanes' keys are never read).
    const uint32_t r1 = static_cast<uint32_t>(r + 1) & 0xffffu;
    const uint32_t rr = r1 | (r1 << 16);
    const uint32_t dlo = tb_sub16x2(static_cast<uint32_t>(c.cum4), rr);
    const uint32_t dhi = tb_sub16x2(static_cast<uint32_t>(c.cum4 >> 32), rr);
    const int fld = static_cast<int>(((dlo >> 15) & 1u) + (dlo >> 31) + ((dhi >> 15) & 1u));
    // cases in the rows before row fld of the lane: C_{fld-1}, 0 for fld 0
    const int before = static_cast<int>(((c.cum4 << 16) >> (16 * fld)) & 0xffffu);
    // (row << 16) | rank in the row
    const int key = ((4 * lane + fld) << 16) | ((r - before) & 0xffff);
    // the last lane whose lower lanes hold at most m cases (lane 0 always);
    // the lane prefixes never decrease, so the lanes after it are those
    // whose lower lanes hold more
    h.after_grp = c.excl > static_cast<int>(m);
    h.grp = 63 - __builtin_clzll(__ballot(!h.after_grp) | 1ull);
    const int k = __builtin_amdgcn_readlane(key, h.grp);
    h.row = k >> 16;
    h.fld = h.row & 3;
    const int rank = k & 0xffff;
    h.pre = pre[64 * h.row + lane];
    // the row's prefixes never decrease either: the slots from col on are
    // those whose prefix exceeds the rank
    h.from_col = h.pre > rank;
    h.col = tb_first(__ballot(h.from_col));
    return h;
}

// Whether slot col of the row held one case before the event: its prefix
// minus the one before it, two lane reads of the row itself (p, this lane's
// prefix before the event).  (The difference formed by a DPP subtract that
// shifts the row by one lane, wave_shr:1, into its own register gave wrong
// counts on gfx950, read either by v_readlane or by a compare.)
__device__ __forceinline__ bool tb_held_one(int p, int col)
{
    const int below = __builtin_amdgcn_readlane(p, (col + 63) & 63);
    return __builtin_amdgcn_readlane(p, col) - (col > 0 ? below : 0) == 1;
}

// Adds d to slot (row, col) whose prefix row this lane holds as p (from_col:
// this lane's slot is col or after it), d cases to the register counts of
// the row in lane grp, and d to the lower-lane counts of the lanes after grp
// (after_grp).
__device__ __forceinline__ void tb_add(uint16_t *pre, TbRegs &c, int grp, int fld, int row, bool from_col,
                                       bool after_grp, int p, int d)
{
    const int lane = threadIdx.x;
    pre[64 * row + lane] = static_cast<uint16_t>(p + (from_col ? d : 0));
    // d to the cumulative counts of rows fld..3 (never below zero: a case
    // leaves only a row that holds it)
    const uint64_t ones = 0x0001000100010001ull;
    const uint64_t dd = (d > 0 ? ones : 0ull - ones) << (16 * fld);
    if (lane == grp)
        c.cum4 += dd;
    c.excl += after_grp ? d : 0;
}

// Adds o occupied slots to the row's register count in lane grp.
__device__ __forceinline__ void tb_occupy(TbRegs &c, int grp, int fld, int o)
{
    const uint64_t od = static_cast<uint64_t>(static_cast<int64_t>(o)) << (16 * fld);
    if (static_cast<int>(threadIdx.x) == grp)
        c.occ4 += od;
}

// A new genotype: one case in the lowest empty slot.
__device__ __forceinline__ void tb_new_genotype(uint16_t *pre, TbRegs &c)
{
    const int lane = threadIdx.x;
    // every lane: its first row that is not full (bit 6 + 16 j of ~occ4)
    const int fld_l = __builtin_ctzll((~c.occ4 & TB_FULL_BITS) | (1ull << 63)) >> 4;
    const int grp = tb_first(__ballot((c.occ4 & TB_FULL_BITS) != TB_FULL_BITS));
    const int row = __builtin_amdgcn_readlane(4 * lane + fld_l, grp);
    const int fld = row & 3;
    const int p = pre[64 * row + lane];
    const int cnt = p - __builtin_amdgcn_update_dpp(0, p, 0x138, 0xF, 0xF, false);
    const int col = tb_first(__ballot(cnt == 0));
    tb_add(pre, c, grp, fld, row, lane >= col, lane > grp, p, 1);
    tb_occupy(c, grp, fld, 1);
}

__global__ __launch_bounds__(TB_BLOCK) void k_simulate_tb(const EpochHeader *__restrict__ hdr,
                                                        const JobDev *__restrict__ rows,
                                                        LaunchState *__restrict__ states)
{
    __shared__ __align__(16) uint16_t s_pre[TB_SLOTS];
    __shared__ float s_samp[PPS_TB_MAX_SAMPLE];
    const int lane = threadIdx.x;
    const int n_jobs = static_cast<int>(hdr->class_rows[CLASS_GILLESPIE]);
    const uint64_t total_tiles = hdr->class_tiles[CLASS_GILLESPIE];
    const JobDev *__restrict__ jobs = rows + hdr->class_first[CLASS_GILLESPIE];
    LaunchState *__restrict__ state = states + CLASS_GILLESPIE;
    // Two passes over the tiles: the first runs the draws whose run is
    // predicted to be long, the second the rest, so that the long runs start
    // at once and the short ones fill the machine around them (the order of
    // the runs changes no result: every draw writes its own outputs).
    for (;;) {
        unsigned long long tl = 0;
        if (lane == 0)
            tl = atomicAdd(&state->next_tile, 1ull);
        const uint64_t t2 = tb_readlane64(tl, 0);
        if (t2 >= 2 * total_tiles)
            break;
        const bool long_pass = t2 < total_tiles;
        const uint64_t t = long_pass ? t2 : t2 - total_tiles;
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const JobDev *__restrict__ J = jobs + lo;
        const int flags = J->flags;
        const uint64_t n = J->n_draws;
        const uint64_t q = t - J->tile_begin + J->tile_offset;  // one draw per tile
        const uint64_t draw = J->first_draw + q;
        const StreamKey key = make_key(J->seed);
        double theta[3];
        prior_draw<3>(J->prior, 3, J->constraint, key, draw, theta);
        const uint32_t n_stop = static_cast<uint32_t>(J->n_cells);
        const uint32_t max_events = static_cast<uint32_t>(J->steps);
        // predicted length: a supercritical run that survives grows at rate
        // (alpha - delta) per case against (alpha + delta + tau) events per
        // case, so it takes about n_stop (alpha + delta + tau)/(alpha - delta)
        // events; long means at least a quarter of the event cap, and runs
        // that are not supercritical count as long
        const double gap = theta[0] - theta[1];
        const bool is_long =
            __builtin_amdgcn_readfirstlane(
                !(gap > 0.0) ||
                static_cast<double>(n_stop) * (theta[0] + theta[1] + theta[2]) >=
                    gap * (static_cast<double>(max_events) * 0.25)) != 0;
        if (is_long != long_pass)
            continue;
        // event-type thresholds: single IEEE FP64 operations (as the oracle),
        // floor(2^32 alpha/R) and floor(2^32 (alpha + delta)/R), at most 2^32
        const double ad = __dadd_rn(theta[0], theta[1]);
        const double rate = __dadd_rn(ad, theta[2]);
        const uint64_t t_birth =
            tb_readlane64(static_cast<uint64_t>(floor(ldexp(__ddiv_rn(theta[0], rate), 32))), 0);
        const uint64_t t_death =
            tb_readlane64(static_cast<uint64_t>(floor(ldexp(__ddiv_rn(ad, rate), 32))), 0);
        // word < threshold as 32-bit compares: a threshold of 2^32 takes every word
        const uint32_t tb32 = static_cast<uint32_t>(min(t_birth, 0xffffffffull));
        const uint32_t td32 = static_cast<uint32_t>(min(t_death, 0xffffffffull));
        const bool b_all = t_birth > 0xffffffffull, d_all = t_death > 0xffffffffull;
        const int nr_used = static_cast<int>((n_stop + 63) / 64);
        // one genotype with x0 cases in slot 0; rows past the population
        // count as full so that no new genotype goes there
        uint32_t N = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(J->x0));
        for (int i = lane; i < nr_used * 64; i += TB_BLOCK)
            s_pre[i] = i < 64 ? static_cast<uint16_t>(N) : 0;
        TbRegs c;
        c.cum4 = lane == 0 ? 0x0001000100010001ull * N : 0;
        c.occ4 = lane == 0 ? 1 : 0;
        c.excl = lane == 0 ? 0 : static_cast<int>(N);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (4 * lane + k >= nr_used)
                c.occ4 |= 64ull << (16 * k);
        __syncthreads();
        uint32_t e = 0;
        // one event: case word wc, the population step dn (+1 birth, -1
        // death, 0 mutation) and the chosen slot's step d (+1 birth, -1
        // otherwise); both are wave-uniform, so N stays scalar
        auto event = [&](uint32_t wc, int dn, int d) {
            const uint32_t m = __umulhi(wc, N);
            const TbHit h = tb_find(s_pre, c, m);
            tb_add(s_pre, c, h.grp, h.fld, h.row, h.from_col, h.after_grp, h.pre, d);
            N += static_cast<uint32_t>(dn);
            if (dn <= 0) {
                // a case left the slot: it is empty now if it held one
                if (tb_held_one(h.pre, h.col))
                    tb_occupy(c, h.grp, h.fld, -1);
                if (dn == 0) {
                    // mutation: the case leaves its genotype for a new one
                    // in the lowest empty slot (after the parent's count
                    // dropped)
                    __builtin_amdgcn_wave_barrier();
                    tb_new_genotype(s_pre, c);
                }
            }
            __builtin_amdgcn_wave_barrier();
        };
        // running: 0 < N < n_stop and e < max_events
        auto running = [&]() { return N - 1 < n_stop - 1 && e < max_events; };
        while (running()) {
            // events e .. e + 127: block e/2 + j in lane j (e is a multiple
            // of 128 here); lane j's type words are those of events e + 2j
            // (word y) and e + 2j + 1 (word w)
            const Words4 wv = stream_block(key, draw, (e >> 1) + static_cast<uint32_t>(lane),
                                           PURPOSE_TB_EVENT);
            const int dn_y = (b_all || wv.y < tb32) ? 1 : ((d_all || wv.y < td32) ? -1 : 0);
            const int dn_w = (b_all || wv.w < tb32) ? 1 : ((d_all || wv.w < td32) ? -1 : 0);
            const int d_y = dn_y > 0 ? 1 : -1, d_w = dn_w > 0 ? 1 : -1;
            int j = 0;
            while (j < 64 && running()) {
                // N moves by at most one per event, so with s = min(N - 1,
                // n_stop - 1 - N) the next s events cannot end the run: they
                // go in pairs without the stop test
                const uint32_t s = min(N - 1, n_stop - 1 - N);
                const int pairs = static_cast<int>(
                    min(min(s >> 1, static_cast<uint32_t>(64 - j)), (max_events - e) >> 1));
                for (int i = 0; i < pairs; ++i, ++j) {
                    event(__builtin_amdgcn_readlane(wv.x, j), __builtin_amdgcn_readlane(dn_y, j),
                          __builtin_amdgcn_readlane(d_y, j));
                    event(__builtin_amdgcn_readlane(wv.z, j), __builtin_amdgcn_readlane(dn_w, j),
                          __builtin_amdgcn_readlane(d_w, j));
                }
                e += 2u * static_cast<uint32_t>(pairs);
                if (pairs == 0) {
                    // near a bound: one pair with the test after each event
                    event(__builtin_amdgcn_readlane(wv.x, j), __builtin_amdgcn_readlane(dn_y, j),
                          __builtin_amdgcn_readlane(d_y, j));
                    ++e;
                    if (!running())
                        break;
                    event(__builtin_amdgcn_readlane(wv.z, j), __builtin_amdgcn_readlane(dn_w, j),
                          __builtin_amdgcn_readlane(d_w, j));
                    ++e;
                    ++j;
                }
            }
        }
        __syncthreads();
        const int32_t status = N >= n_stop ? TB_COMPLETE : (N == 0 ? TB_EXTINCT : TB_TRUNCATED);
        // summaries: n_sample cases without replacement (all when fewer)
        const uint32_t n_sample = static_cast<uint32_t>(J->n_sample);
        uint64_t g = 0, sq = 0, n_taken = 0;
        if (N >= n_sample) {
            n_taken = n_sample;
            // sample s: word s%4 of block s/4; 64 blocks (256 samples) at a time
            for (uint32_t s0 = 0; s0 < n_sample; s0 += 256) {
                const Words4 ws = stream_block(key, draw, (s0 >> 2) + static_cast<uint32_t>(lane),
                                               PURPOSE_TB_SAMPLE);
                const uint32_t s_end = min(n_sample, s0 + 256);
                for (uint32_t si = s0; si < s_end; ++si) {
                    const int j = static_cast<int>((si - s0) >> 2);
                    const int wsel = static_cast<int>(si & 3);
                    const uint32_t wv = __builtin_amdgcn_readlane(
                        wsel == 0 ? ws.x : (wsel == 1 ? ws.y : (wsel == 2 ? ws.z : ws.w)), j);
                    const TbHit h = tb_find(s_pre, c, __umulhi(wv, N - si));
                    tb_add(s_pre, c, h.grp, h.fld, h.row, h.from_col, h.after_grp, h.pre, -1);
                    if (lane == 0)
                        s_samp[si] = static_cast<float>(64 * h.row + h.col);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            unsigned n2 = 1;
            while (n2 < n_sample)
                n2 <<= 1;
            for (unsigned i = n_sample + lane; i < n2; i += TB_BLOCK)
                s_samp[i] = __builtin_inff();
            __syncthreads();
            lds_bitonic_sort<TB_BLOCK>(s_samp, n2);
            // runs of equal slots: g runs, sum of squared run lengths (every
            // lane walks the sorted slots: broadcast reads, uniform control)
            uint64_t run = 0;
            float prev = -1.0f;
            for (uint32_t i = 0; i < n_sample; ++i) {
                const float v = s_samp[i];
                if (v != prev) {
                    sq += run * run;
                    run = 0;
                    ++g;
                    prev = v;
                }
                ++run;
            }
            sq += run * run;
        } else if (N > 0) {
            n_taken = N;
            uint64_t gl = 0, sl = 0;
            for (int r = 0; r < nr_used; ++r) {
                const int p = s_pre[64 * r + lane];
                const uint64_t v = static_cast<uint32_t>(
                    p - __builtin_amdgcn_update_dpp(0, p, 0x138, 0xF, 0xF, false));
                gl += v > 0;
                sl += v * v;
            }
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                gl += __shfl_xor(gl, d, 64);
                sl += __shfl_xor(sl, d, 64);
            }
            g = gl;
            sq = sl;
        }
        double s0 = 0.0, s1 = 0.0;
        if (n_taken > 0) {
            const double nt = static_cast<double>(n_taken);
            s0 = static_cast<double>(g) / nt;
            s1 = 1.0 - static_cast<double>(sq) / (nt * nt);
        }
        if (lane == 0) {
            if ((flags & JOB_EVENTS) && J->dump_events)
                J->dump_events[q] = e;
            if ((flags & JOB_EVENTS) && J->dump_status)
                J->dump_status[q] = status;
            const double d0 = s0 - static_cast<double>(J->y_obs[0]);
            const double d1 = s1 - static_cast<double>(J->y_obs[1]);
            const float dist = static_cast<float>(sqrt(d0 * d0 + d1 * d1));
            const double stat = 0.5 * (s0 + s1);
            if (flags & JOB_WRITE_DIST)
                J->dist[q] = dist;
            if (flags & JOB_DUMP) {
                if (J->dump_theta) {
                    J->dump_theta[q] = static_cast<float>(theta[0]);
                    J->dump_theta[n + q] = static_cast<float>(theta[1]);
                    J->dump_theta[2 * n + q] = static_cast<float>(theta[2]);
                }
                if (J->dump_summ) {
                    J->dump_summ[q] = static_cast<float>(s0);
                    J->dump_summ[n + q] = static_cast<float>(s1);
                }
                if (J->dump_stat)
                    J->dump_stat[q] = static_cast<float>(stat);
                if (J->dump_dist)
                    J->dump_dist[q] = dist;
            }
            if (flags & JOB_TALLY_SUMM) {
                if (s0 >= J->summ_obs[0])
                    atomicAdd(&J->counts[0], 1ull);
                if (s1 >= J->summ_obs[1])
                    atomicAdd(&J->counts[1], 1ull);
            }
            if ((flags & JOB_TALLY_STAT) && stat >= J->t_obs)
                atomicAdd(&J->counts[0], 1ull);
        }
        __syncthreads();
    }
}

// ===========================================================================
// Epoch staging: tables in, results out (mapped pinned host memory).
// ===========================================================================
__global__ void k_stage_in(const EpochHeader *__restrict__ h_hdr, const JobDev *__restrict__ h_rows,
                           const FinJob *__restrict__ h_fins, EpochHeader *__restrict__ d_hdr,
                           JobDev *__restrict__ d_rows, FinJob *__restrict__ d_fins,
                           LaunchState *__restrict__ states)
{
    const uint32_t n_rows = h_hdr->n_rows;
    const uint32_t n_fins = h_hdr->n_fins;
    const uint64_t gtid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t gsize = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    const uint64_t row_words = n_rows * (sizeof(JobDev) / sizeof(uint4));
    const uint64_t fin_words = n_fins * (sizeof(FinJob) / sizeof(uint4));
    const uint4 *src_r = reinterpret_cast<const uint4 *>(h_rows);
    uint4 *dst_r = reinterpret_cast<uint4 *>(d_rows);
    for (uint64_t i = gtid; i < row_words; i += gsize)
        dst_r[i] = src_r[i];
    const uint4 *src_f = reinterpret_cast<const uint4 *>(h_fins);
    uint4 *dst_f = reinterpret_cast<uint4 *>(d_fins);
    for (uint64_t i = gtid; i < fin_words; i += gsize)
        dst_f[i] = src_f[i];
    for (uint64_t r = gtid; r < n_rows; r += gsize) {
        if (h_rows[r].row_flags & ROW_ZERO_COUNTS) {
            unsigned long long *c = h_rows[r].counts;
            for (uint32_t s = 0; s < h_rows[r].n_counts; ++s)
                c[s] = 0ull;
        }
    }
    if (gtid == 0) {
        *d_hdr = *h_hdr;
        for (int c = 0; c < N_CLASSES; ++c)
            states[c].next_tile = 0ull;
    }
}

__global__ void k_stage_out(const EpochHeader *__restrict__ d_hdr, const JobDev *__restrict__ d_rows,
                            const FinJob *__restrict__ d_fins, FinResult *__restrict__ h_out_fin,
                            unsigned long long *__restrict__ h_out_counts)
{
    const uint32_t n_rows = d_hdr->n_rows;
    const uint32_t n_fins = d_hdr->n_fins;
    const uint64_t gtid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t gsize = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = gtid; i < n_fins; i += gsize)
        h_out_fin[i] = *d_fins[i].result;
    for (uint64_t r = gtid; r < n_rows; r += gsize) {
        const JobDev &R = d_rows[r];
        if (R.row_flags & ROW_COPY_COUNTS)
            for (uint32_t s = 0; s < R.n_counts; ++s)
                h_out_counts[R.out_slot + s] = R.counts[s];
    }
}

// ===========================================================================
// Random-stream dumps.
// ===========================================================================
__global__ void k_philox(uint64_t seed, uint64_t first, uint64_t n, uint32_t block,
                         uint32_t purpose, uint32_t *__restrict__ out)
{
    const StreamKey key = make_key(seed);
    for (uint64_t q = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; q < n;
         q += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const Words4 w = stream_block(key, first + q, block, purpose);
        uint4 v;
        v.x = w.x;
        v.y = w.y;
        v.z = w.z;
        v.w = w.w;
        reinterpret_cast<uint4 *>(out)[q] = v;
    }
}

__global__ void k_normals(uint64_t seed, uint64_t first, uint64_t n, uint32_t m,
                          float *__restrict__ out)
{
    const StreamKey key = make_key(seed);
    for (uint64_t q = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; q < n;
         q += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        for (uint32_t b = 0; NORMALS_PER_BLOCK * b < m; ++b) {
            float z[NORMALS_PER_BLOCK];
            path_normals6(key, first + q, b, z);
            for (uint32_t j = 0; j < NORMALS_PER_BLOCK && NORMALS_PER_BLOCK * b + j < m; ++j)
                out[static_cast<uint64_t>(NORMALS_PER_BLOCK * b + j) * n + q] = z[j];
        }
    }
}

// ===========================================================================
// ABC finalisation.  Per-element kernels loop over the epoch's finalisation
// blocks with a fixed grid; per-job kernels run one workgroup per job with
// grid MAX_FINS (surplus workgroups exit).  Fixed grids keep the epoch
// graph's shape independent of the jobs it carries.
// ===========================================================================
__device__ __forceinline__ int fin_locate(const FinJob *__restrict__ fins, int n_fins, uint64_t b)
{
    int lo = 0, hi = n_fins - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fins[mid].block_begin <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void sel_digit(int pass, int &shift, int &bits)
{
    if (pass == 0) {
        shift = 32 - SEL_BITS0;
        bits = SEL_BITS0;
    } else if (pass == 1) {
        shift = 32 - SEL_BITS0 - SEL_BITS1;
        bits = SEL_BITS1;
    } else {
        shift = 0;
        bits = SEL_BITS2;
    }
}

// One workgroup per job: reset the select state and zero the histogram.
__global__ __launch_bounds__(FIN_BLOCK) void k_fin_init(const EpochHeader *__restrict__ hdr,
                                                         const FinJob *__restrict__ fins)
{
    if (blockIdx.x >= hdr->n_fins)
        return;
    const FinJob *F = fins + blockIdx.x;
    for (int i = threadIdx.x; i < SEL_BINS; i += FIN_BLOCK)
        F->hist[i] = 0;
    if (threadIdx.x == 0) {
        FinResult *R = F->result;
        R->sel_prefix = 0;
        R->sel_mask = 0;
        R->sel_rank = F->k;
        R->thresh_bits = 0;
        R->quota = 0;
        R->lt_total = 0;
        R->eq_total = 0;
        R->n_accepted = 0;
    }
}

__global__ __launch_bounds__(FIN_BLOCK) void k_sel_hist(const EpochHeader *__restrict__ hdr,
                                                         const FinJob *__restrict__ fins, int pass)
{
    __shared__ unsigned h[SEL_BINS];
    if (!hdr->any_top)
        return;
    const int n_fins = static_cast<int>(hdr->n_fins);
    const uint64_t total = hdr->fin_blocks;
    int shift, bits;
    sel_digit(pass, shift, bits);
    const uint32_t dmask = (1u << bits) - 1u;
    for (uint64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const FinJob *F = fins + fin_locate(fins, n_fins, b);
        if (F->mode != PPS_EPS_TOP_FRACTION)
            continue;  // uniform across the workgroup
        const uint32_t prefix = F->result->sel_prefix;
        const uint32_t pmask = F->result->sel_mask;
        for (int i = threadIdx.x; i < SEL_BINS; i += FIN_BLOCK)
            h[i] = 0;
        __syncthreads();
        const uint64_t base = (b - F->block_begin) * static_cast<uint64_t>(FIN_TILE);
        const uint32_t *__restrict__ d = reinterpret_cast<const uint32_t *>(F->dist);
        const uint64_t n = F->n;
        // all rows' loads in flight before the first histogram update
        uint32_t dv[FIN_ROWS];
#pragma unroll
        for (int r = 0; r < FIN_ROWS; ++r) {
            const uint64_t e = base + static_cast<uint64_t>(r) * FIN_BLOCK + threadIdx.x;
            dv[r] = e < n ? d[e] : 0u;
        }
#pragma unroll
        for (int r = 0; r < FIN_ROWS; ++r) {
            const uint64_t e = base + static_cast<uint64_t>(r) * FIN_BLOCK + threadIdx.x;
            if (e < n && (dv[r] & pmask) == prefix)
                atomicAdd(&h[(dv[r] >> shift) & dmask], 1u);
        }
        __syncthreads();
        for (int i = threadIdx.x; i <= static_cast<int>(dmask); i += FIN_BLOCK)
            if (h[i])
                atomicAdd(&F->hist[i], h[i]);
        __syncthreads();
    }
}

// One workgroup per job: find the digit holding the rank still sought.
__global__ __launch_bounds__(FIN_BLOCK) void k_sel_pick(const EpochHeader *__restrict__ hdr,
                                                         const FinJob *__restrict__ fins, int pass)
{
    __shared__ unsigned long long s_sum[FIN_BLOCK];
    if (!hdr->any_top || blockIdx.x >= hdr->n_fins)
        return;
    const FinJob *F = fins + blockIdx.x;
    if (F->mode != PPS_EPS_TOP_FRACTION)
        return;
    FinResult *R = F->result;
    int shift, bits;
    sel_digit(pass, shift, bits);
    const int nb = 1 << bits;
    const int per = nb / FIN_BLOCK;  // 8 or 4 bins per thread
    const int b0 = threadIdx.x * per;
    unsigned long long local = 0;
    for (int i = 0; i < per; ++i)
        local += F->hist[b0 + i];
    s_sum[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < FIN_BLOCK; off <<= 1) {
        const unsigned long long v = threadIdx.x >= off ? s_sum[threadIdx.x - off] : 0ull;
        __syncthreads();
        s_sum[threadIdx.x] += v;
        __syncthreads();
    }
    const uint64_t rank = R->sel_rank;
    const unsigned long long incl = s_sum[threadIdx.x];
    const unsigned long long before = incl - local;
    __syncthreads();
    if (before < rank && rank <= incl) {
        unsigned long long cum = before;
        for (int i = 0; i < per; ++i) {
            const unsigned c = F->hist[b0 + i];
            if (cum + c >= rank) {
                R->sel_prefix |= static_cast<uint32_t>(b0 + i) << shift;
                R->sel_mask |= static_cast<uint32_t>(nb - 1) << shift;
                R->sel_rank = rank - cum;
                break;
            }
            cum += c;
        }
    }
    __syncthreads();
    for (int i = 0; i < per; ++i)
        F->hist[b0 + i] = 0;
    if (pass == 2 && threadIdx.x == 0) {
        __threadfence_block();
        R->thresh_bits = R->sel_prefix;
        R->quota = R->sel_rank;
    }
}

// A wave's FIN_ROWS distances (rows of 64 from wbase), loaded before any of
// them is used so that the loads are in flight together; past n reads 0.
__device__ __forceinline__ void fin_rows(const float *__restrict__ dist, uint64_t n, uint64_t wbase,
                                         float (&dv)[FIN_ROWS])
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int r = 0; r < FIN_ROWS; ++r) {
        const uint64_t e = wbase + static_cast<uint64_t>(r) * 64 + lane;
        dv[r] = e < n ? dist[e] : 0.0f;
    }
}

// fin_pred on a loaded distance (valid: the element is below n).
__device__ __forceinline__ void fin_pred_d(int mode, double eps, uint32_t thresh, bool valid, float d,
                                           bool &lt, bool &eq)
{
    if (mode == PPS_EPS_FIXED) {
        lt = valid && static_cast<double>(d) <= eps;
        eq = false;
    } else {
        const uint32_t v = __float_as_uint(d);
        lt = valid && v < thresh;
        eq = valid && v == thresh;
    }
}

// Per block: (count rho "below", count "tied") over its FIN_TILE elements.
__global__ __launch_bounds__(FIN_BLOCK) void k_compact_count(const EpochHeader *__restrict__ hdr,
                                                              const FinJob *__restrict__ fins)
{
    __shared__ unsigned s_lt[FIN_BLOCK / 64], s_eq[FIN_BLOCK / 64];
    const int n_fins = static_cast<int>(hdr->n_fins);
    const uint64_t total = hdr->fin_blocks;
    const int wave = threadIdx.x >> 6;
    for (uint64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const FinJob *F = fins + fin_locate(fins, n_fins, b);
        const uint64_t lb = b - F->block_begin;
        const uint32_t thresh = F->result->thresh_bits;
        const uint64_t n = F->n;
        const int mode = F->mode;
        const double eps = F->eps;
        const uint64_t wbase = lb * FIN_TILE + static_cast<uint64_t>(wave) * (FIN_ROWS * 64);
        float dv[FIN_ROWS];
        fin_rows(F->dist, n, wbase, dv);
        unsigned clt = 0, ceq = 0;
#pragma unroll
        for (int r = 0; r < FIN_ROWS; ++r) {
            bool lt, eq;
            fin_pred_d(mode, eps, thresh, wbase + r * 64 + lane_id() < n, dv[r], lt, eq);
            clt += __popcll(__ballot(lt));
            ceq += __popcll(__ballot(eq));
        }
        if (lane_id() == 0) {
            s_lt[wave] = clt;
            s_eq[wave] = ceq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long a = 0, c = 0;
            for (int w = 0; w < FIN_BLOCK / 64; ++w) {
                a += s_lt[w];
                c += s_eq[w];
            }
            F->block_counts[2 * lb] = a;
            F->block_counts[2 * lb + 1] = c;
        }
        __syncthreads();
    }
}

// One workgroup per job: exclusive scan of the per-block (lt, eq) counts.
// Thread t owns the consecutive blocks [t c, (t + 1) c): it sums them (loads
// independent of each other), the workgroup scans the 256 sums once, and the
// thread rewrites its blocks as running offsets from its scanned start.
__global__ __launch_bounds__(FIN_BLOCK) void k_compact_scan(const EpochHeader *__restrict__ hdr,
                                                             const FinJob *__restrict__ fins)
{
    __shared__ unsigned long long s_a[FIN_BLOCK], s_b[FIN_BLOCK];
    if (blockIdx.x >= hdr->n_fins)
        return;
    const FinJob *F = fins + blockIdx.x;
    FinResult *R = F->result;
    const uint64_t nb = F->n_blocks;
    const uint64_t chunk = (nb + FIN_BLOCK - 1) / FIN_BLOCK;
    const uint64_t b0 = threadIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < nb ? b0 + chunk : nb;
    unsigned long long *__restrict__ bc = F->block_counts;
    unsigned long long sa = 0, sb = 0;
    for (uint64_t i = b0; i < b1; ++i) {
        sa += bc[2 * i];
        sb += bc[2 * i + 1];
    }
    s_a[threadIdx.x] = sa;
    s_b[threadIdx.x] = sb;
    __syncthreads();
    for (int off = 1; off < FIN_BLOCK; off <<= 1) {
        const unsigned long long va = threadIdx.x >= off ? s_a[threadIdx.x - off] : 0ull;
        const unsigned long long vb = threadIdx.x >= off ? s_b[threadIdx.x - off] : 0ull;
        __syncthreads();
        s_a[threadIdx.x] += va;
        s_b[threadIdx.x] += vb;
        __syncthreads();
    }
    unsigned long long ra = s_a[threadIdx.x] - sa, rb = s_b[threadIdx.x] - sb;
    for (uint64_t i = b0; i < b1; ++i) {
        const unsigned long long a = bc[2 * i], b = bc[2 * i + 1];
        bc[2 * i] = ra;
        bc[2 * i + 1] = rb;
        ra += a;
        rb += b;
    }
    const unsigned long long carry_a = s_a[FIN_BLOCK - 1], carry_b = s_b[FIN_BLOCK - 1];
    if (threadIdx.x == 0) {
        R->lt_total = carry_a;
        R->eq_total = carry_b;
        const uint64_t take = F->mode == PPS_EPS_FIXED ? 0 : (carry_b < R->quota ? carry_b : R->quota);
        R->n_accepted = carry_a + take;
        R->eps_used = F->mode == PPS_EPS_FIXED ? F->eps
                                               : static_cast<double>(__uint_as_float(R->thresh_bits));
    }
}

struct Moments {
    double n;
    double mean[PPS_MAX_PARAMS];
    double m2[PPS_MAX_PARAMS];
};

// Chan et al. pairwise update: a <- a (+) b (a first in index order).
// Branch-free: an empty side (n = 0, zero mean and m2) leaves the other
// exactly as it is (weights 0 or 1), so the result equals the form that
// copies or skips, and the loads of b are never made conditional on b.n.
__device__ __forceinline__ void moments_merge(Moments &a, const Moments &b, int np)
{
    const double n = a.n + b.n;
    const double wb = n > 0.0 ? b.n / n : 0.0;
    const double wab = n > 0.0 ? a.n * b.n / n : 0.0;
#pragma unroll
    for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
        if (j < np) {
            const double delta = b.mean[j] - a.mean[j];
            a.mean[j] += delta * wb;
            a.m2[j] += b.m2[j] + delta * delta * wab;
        }
    }
    a.n = n;
}

// The same result, skipping the arithmetic when a side is empty: cheaper
// where most operands are empty (the tail of a small job's fold tree);
// elsewhere the branch-free form keeps the instruction stream free of waits
// on the operands.
__device__ __forceinline__ void moments_merge_skip(Moments &a, const Moments &b, int np)
{
    if (b.n == 0.0)
        return;
    if (a.n == 0.0) {
        a = b;
        return;
    }
    moments_merge(a, b, np);
}

__device__ __forceinline__ double moments_readlane(double v, int l)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(b), l);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(b >> 32), l);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

constexpr int PARTIAL_STRIDE = 1 + 2 * PPS_MAX_PARAMS;
constexpr unsigned MOMENTS_GRID = 256;  // workgroups of k_moments_final

// Writes accepted records in draw-index order and per-block moment partials.
__global__ __launch_bounds__(FIN_BLOCK) void k_compact_write(const EpochHeader *__restrict__ hdr,
                                                              const FinJob *__restrict__ fins)
{
    constexpr int NW = FIN_BLOCK / 64;
    __shared__ unsigned s_lt[NW], s_eq[NW];
    __shared__ Moments s_mom[NW];
    // each wave's distances for the second pass (each lane reads back only
    // what it wrote, so no barrier is needed)
    __shared__ float s_dv[NW][FIN_ROWS][64];
    // per wave: accepted draws waiting for their records (tile offset and
    // record position); at most 63 + 64 at once
    __shared__ uint16_t s_qoff[NW][128];
    __shared__ uint64_t s_qpos[NW][128];
    const int n_fins = static_cast<int>(hdr->n_fins);
    const uint64_t total = hdr->fin_blocks;
    const int wave = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const FinJob *F = fins + fin_locate(fins, n_fins, b);
        const FinResult *R = F->result;
        const uint64_t lb = b - F->block_begin;
        const uint32_t thresh = R->thresh_bits;
        const uint64_t quota = F->mode == PPS_EPS_FIXED ? 0 : R->quota;
        const uint64_t wbase = lb * FIN_TILE + static_cast<uint64_t>(wave) * (FIN_ROWS * 64);
        const int np = F->n_params;
        // the job's fields in registers (the record stores below could
        // otherwise alias them and force reloads)
        const uint64_t n = F->n;
        const int mode = F->mode;
        const double eps = F->eps;
        const uint64_t first = F->first_draw, capacity = F->capacity;
        uint64_t *__restrict__ acc_idx = F->acc_idx;
        float *__restrict__ acc_dist = F->acc_dist;
        float *__restrict__ acc_theta = F->acc_theta;
        float dv[FIN_ROWS];
        fin_rows(F->dist, n, wbase, dv);
        // pass 1: this wave's totals, for the prefix over the block's waves
        unsigned clt = 0, ceq = 0;
#pragma unroll
        for (int r = 0; r < FIN_ROWS; ++r) {
            bool lt, eq;
            fin_pred_d(mode, eps, thresh, wbase + r * 64 + lane < n, dv[r], lt, eq);
            clt += __popcll(__ballot(lt));
            ceq += __popcll(__ballot(eq));
            s_dv[wave][r][lane] = dv[r];
        }
        if (lane == 0) {
            s_lt[wave] = clt;
            s_eq[wave] = ceq;
        }
        __syncthreads();
        uint64_t lt_before = F->block_counts[2 * lb];
        uint64_t eq_before = F->block_counts[2 * lb + 1];
        for (int w = 0; w < wave; ++w) {
            lt_before += s_lt[w];
            eq_before += s_eq[w];
        }
        Moments mom;
        mom.n = 0.0;
#pragma unroll
        for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
            mom.mean[j] = 0.0;
            mom.m2[j] = 0.0;
        }
        const StreamKey key = make_key(F->seed);
        // Accepted draws of queue slots [0, k): lane l < k takes slot l,
        // recomputes its theta from the stream, writes the record and adds
        // it to its running moments (lane l sees slots l, 64 + l, ... of the
        // wave's accepted draws: a fixed order).
        auto flush = [&](int k) {
            // the queue slots were written by other lanes of this wave: LDS
            // operations of one wave complete in order, and this keeps the
            // compiler from moving them
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (static_cast<int>(lane) < k) {
                const uint32_t off = s_qoff[wave][lane];
                const uint64_t pos = s_qpos[wave][lane];
                const uint64_t e = wbase + off;
                double theta[PPS_MAX_PARAMS];
                prior_draw<PPS_MAX_PARAMS>(F->prior, np, F->constraint, key, first + e, theta);
                if (pos < capacity) {
                    acc_idx[pos] = first + e;
                    acc_dist[pos] = s_dv[wave][off >> 6][off & 63];
#pragma unroll
                    for (int j = 0; j < PPS_MAX_PARAMS; ++j)
                        if (j < np)
                            acc_theta[static_cast<uint64_t>(j) * capacity + pos] =
                                static_cast<float>(theta[j]);
                }
                // Welford update
                mom.n += 1.0;
                const double inv_n = 1.0 / mom.n;
#pragma unroll
                for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
                    if (j < np) {
                        const double delta = theta[j] - mom.mean[j];
                        mom.mean[j] += delta * inv_n;
                        mom.m2[j] += delta * (theta[j] - mom.mean[j]);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        // pass 2: ranks; accepted draws queue up in index order and are
        // written 64 at a time, so that the prior recomputation (three Philox
        // calls and FP64 work per draw) runs on whole waves rather than once
        // per row for its one or two accepted lanes
        int q = 0;  // queue length (wave-uniform, below 64 between rows)
        for (int r = 0; r < FIN_ROWS; ++r) {
            const uint64_t e = wbase + r * 64 + lane;
            bool lt, eq;
            const float d = s_dv[wave][r][lane];
            fin_pred_d(mode, eps, thresh, e < n, d, lt, eq);
            const uint64_t mlt = __ballot(lt);
            const uint64_t meq = __ballot(eq);
            if (mlt | meq) {
                const uint64_t my_lt = lt_before + __popcll(mlt & below);
                const uint64_t my_eq = eq_before + __popcll(meq & below);
                const bool acc = lt || (eq && my_eq < quota);
                const uint64_t macc = __ballot(acc);
                if (acc) {
                    const int slot = q + __popcll(macc & below);
                    s_qoff[wave][slot] = static_cast<uint16_t>(r * 64 + lane);
                    s_qpos[wave][slot] = my_lt + (my_eq < quota ? my_eq : quota);
                }
                q += __popcll(macc);
                lt_before += __popcll(mlt);
                eq_before += __popcll(meq);
                if (q >= 64) {
                    flush(64);
                    q -= 64;
                    // the rest (fewer than 64) moves to the queue's front
                    uint16_t off = 0;
                    uint64_t pos = 0;
                    if (static_cast<int>(lane) < q) {
                        off = s_qoff[wave][64 + lane];
                        pos = s_qpos[wave][64 + lane];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    if (static_cast<int>(lane) < q) {
                        s_qoff[wave][lane] = off;
                        s_qpos[wave][lane] = pos;
                    }
                }
            }
        }
        if (q > 0)
            flush(q);
        // lanes -> wave: the lanes holding accepted draws (usually none or
        // one: acceptance is rare), merged in lane order; waves -> block
        Moments wm;
        wm.n = 0.0;
#pragma unroll
        for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
            wm.mean[j] = 0.0;
            wm.m2[j] = 0.0;
        }
        for (unsigned long long has = __ballot(mom.n > 0.0); has != 0; has &= has - 1) {
            const int l = __builtin_ctzll(has);
            Moments o;
            o.n = moments_readlane(mom.n, l);
#pragma unroll
            for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
                o.mean[j] = moments_readlane(mom.mean[j], l);
                o.m2[j] = moments_readlane(mom.m2[j], l);
            }
            moments_merge(wm, o, np);
        }
        if (lane == 0)
            s_mom[wave] = wm;
        __syncthreads();
        if (threadIdx.x == 0) {
            Moments acc = s_mom[0];
            for (int w = 1; w < NW; ++w)
                moments_merge(acc, s_mom[w], np);
            double *p = F->partials + lb * PARTIAL_STRIDE;
            p[0] = acc.n;
#pragma unroll
            for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
                p[1 + j] = acc.mean[j];
                p[1 + PPS_MAX_PARAMS + j] = acc.m2[j];
            }
        }
        __syncthreads();
    }
}

// One workgroup per job: fold the per-block partials in block order.
__global__ __launch_bounds__(FIN_BLOCK) void k_moments_final(const EpochHeader *__restrict__ hdr,
                                                              const FinJob *__restrict__ fins)
{
    __shared__ Moments s_m[FIN_BLOCK];
    const int n_fins = static_cast<int>(hdr->n_fins);
    for (int f = blockIdx.x; f < n_fins; f += gridDim.x) {
        const FinJob *F = fins + f;
        FinResult *R = F->result;
        const int np = F->n_params;
        const uint64_t nb = F->n_blocks;
        const uint64_t chunk = (nb + FIN_BLOCK - 1) / FIN_BLOCK;
        Moments m;
        m.n = 0.0;
#pragma unroll
        for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
            m.mean[j] = 0.0;
            m.m2[j] = 0.0;
        }
        // this thread's partials in block order, loaded four at a time
        // before their merges (one memory round trip per four partials)
        const uint64_t b_end = (threadIdx.x + 1) * chunk < nb ? (threadIdx.x + 1) * chunk : nb;
        for (uint64_t b0 = threadIdx.x * chunk; b0 < b_end; b0 += 4) {
            Moments o[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t b = b0 + u < b_end ? b0 + u : b0;
                const double *__restrict__ p = F->partials + b * PARTIAL_STRIDE;
                o[u].n = p[0];
#pragma unroll
                for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
                    o[u].mean[j] = p[1 + j];
                    o[u].m2[j] = p[1 + PPS_MAX_PARAMS + j];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (b0 + u < b_end)
                    moments_merge(m, o[u], np);
        }
        s_m[threadIdx.x] = m;
        __syncthreads();
        for (int off = 1; off < FIN_BLOCK; off <<= 1) {
            if ((threadIdx.x & (2 * off - 1)) == 0 && threadIdx.x + off < FIN_BLOCK)
                moments_merge_skip(s_m[threadIdx.x], s_m[threadIdx.x + off], np);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const Moments &t = s_m[0];
            const double nan = __longlong_as_double(0x7ff8000000000000ll);
            for (int j = 0; j < PPS_MAX_PARAMS; ++j) {
                R->mean[j] = (j < np && t.n > 0.0) ? t.mean[j] : nan;
                R->var[j] = (j < np && t.n > 1.0) ? t.m2[j] / (t.n - 1.0) : nan;
            }
        }
        __syncthreads();  // s_m is reused by the next job
    }
}

// ===========================================================================
// Host-side launchers.
// ===========================================================================
static inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap)
{
    uint64_t g = (n + block - 1) / block;
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return static_cast<unsigned>(g);
}

using SimKernel = void (*)(const EpochHeader *, const JobDev *, LaunchState *);

template <int BLOCK, int CLASS, int DPL, int UNROLL>
static SimKernel sim_ptr()
{
    return k_simulate<BLOCK, CLASS, DPL, UNROLL>;
}

// Kernel instance for a launch shape; null for an unsupported shape.
static SimKernel sim_kernel(int cls, const SimShape &sh)
{
    if (cls == CLASS_GARCH) {
        if (sh.dpl != 1 || sh.unroll != 1)
            return nullptr;
        switch (sh.block) {
        case 64: return sim_ptr<64, CLASS_GARCH, 1, 1>();
        case 128: return sim_ptr<128, CLASS_GARCH, 1, 1>();
        case 256: return sim_ptr<256, CLASS_GARCH, 1, 1>();
        default: return nullptr;
        }
    }
    if (cls == CLASS_CELLS) {
        if (sh.dpl != 1 || sh.unroll != 1)
            return nullptr;
        switch (sh.block) {
        case 256: return k_simulate_cells<256>;
        case 512: return k_simulate_cells<512>;
        case 1024: return k_simulate_cells<1024>;
        default: return nullptr;
        }
    }
    if (cls == CLASS_GILLESPIE)
        return sh.block == TB_BLOCK && sh.dpl == 1 && sh.unroll == 1 ? k_simulate_tb : nullptr;
    if (cls == CLASS_GROUP) {
        if (sh.dpl != 1 || sh.unroll != 1)
            return nullptr;
        switch (sh.block) {
        case 64: return k_simulate_group<64, GROUP_LPL>;
        case 128: return k_simulate_group<128, GROUP_LPL>;
        case 256: return k_simulate_group<256, GROUP_LPL>;
        default: return nullptr;
        }
    }
#define PPS_PATH_SHAPES(B)                                                                         \
    if (sh.block == B) {                                                                           \
        if (sh.dpl == 1 && sh.unroll == 1) return sim_ptr<B, CLASS_PATH, 1, 1>();                  \
        if (sh.dpl == 1 && sh.unroll == 2) return sim_ptr<B, CLASS_PATH, 1, 2>();                  \
        if (sh.dpl == 2 && sh.unroll == 1) return sim_ptr<B, CLASS_PATH, 2, 1>();                  \
        if (sh.dpl == 2 && sh.unroll == 2) return sim_ptr<B, CLASS_PATH, 2, 2>();                  \
        return nullptr;                                                                            \
    }
    PPS_PATH_SHAPES(64)
    PPS_PATH_SHAPES(128)
    PPS_PATH_SHAPES(256)
#undef PPS_PATH_SHAPES
    return nullptr;
}

bool sim_shape_supported(int cls, const SimShape &sh) { return sim_kernel(cls, sh) != nullptr; }

hipError_t sim_occupancy(int cls, const SimShape &sh, int *blocks_per_cu)
{
    SimKernel k = sim_kernel(cls, sh);
    if (!k)
        return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, sh.block, 0);
}

hipError_t issue_epoch_part(int part, const EpochDevPtrs &p, const EpochShape &shape, hipStream_t s)
{
    if (part == EPOCH_STAGE_IN) {
        hipLaunchKernelGGL(k_stage_in, dim3(STAGE_GRID), dim3(256), 0, s, p.h_hdr, p.h_rows,
                           p.h_fins, p.d_hdr, p.d_rows, p.d_fins, p.states);
        return hipGetLastError();
    }
    if (part >= EPOCH_SIMULATE && part < EPOCH_SIMULATE + N_CLASSES) {
        const int c = part - EPOCH_SIMULATE;
        SimKernel k = sim_kernel(c, shape.sim[c]);
        if (!k)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k, dim3(shape.sim_grid[c]), dim3(shape.sim[c].block), 0, s, p.d_hdr,
                           p.d_rows, p.states);
        return hipGetLastError();
    }
    if (part == EPOCH_STAGE_OUT) {
        hipLaunchKernelGGL(k_stage_out, dim3(STAGE_GRID), dim3(256), 0, s, p.d_hdr, p.d_rows,
                           p.d_fins, p.h_out_fin, p.h_out_counts);
        return hipGetLastError();
    }
    if (part != EPOCH_FINALIZE && part != EPOCH_FINALIZE_FIXED)
        return hipErrorInvalidValue;
    const dim3 fb(FIN_BLOCK);
    hipLaunchKernelGGL(k_fin_init, dim3(MAX_FINS), fb, 0, s, p.d_hdr, p.d_fins);
    if (part == EPOCH_FINALIZE)
        for (int pass = 0; pass < 3; ++pass) {
            hipLaunchKernelGGL(k_sel_hist, dim3(shape.fin_grid), fb, 0, s, p.d_hdr, p.d_fins, pass);
            hipLaunchKernelGGL(k_sel_pick, dim3(MAX_FINS), fb, 0, s, p.d_hdr, p.d_fins, pass);
        }
    hipLaunchKernelGGL(k_compact_count, dim3(shape.fin_grid), fb, 0, s, p.d_hdr, p.d_fins);
    hipLaunchKernelGGL(k_compact_scan, dim3(MAX_FINS), fb, 0, s, p.d_hdr, p.d_fins);
    hipLaunchKernelGGL(k_compact_write, dim3(shape.fin_grid), fb, 0, s, p.d_hdr, p.d_fins);
    // few workgroups, each taking jobs in turn: the kernel holds many
    // registers, and surplus workgroups of a MAX_FINS grid cost a dispatch
    // round of their own
    hipLaunchKernelGGL(k_moments_final, dim3(MOMENTS_GRID), fb, 0, s, p.d_hdr, p.d_fins);
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, uint64_t first, uint64_t n, uint32_t block,
                         uint32_t purpose, uint32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_philox, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, seed, first, n,
                       block, purpose, out);
    return hipGetLastError();
}

hipError_t launch_normals(uint64_t seed, uint64_t first, uint64_t n, uint32_t m, float *out,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_normals, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, seed, first, n,
                       m, out);
    return hipGetLastError();
}

}  // namespace pps
