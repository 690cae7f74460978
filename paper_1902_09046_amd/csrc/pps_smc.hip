// Weak-informativity test on gfx950 (Sec. 4.1): data sets of the dose-response
// model of Eq. bioassay, the adaptive SMC evidence estimator of Alg. 3 with
// one sampler per workgroup and one particle per lane (FP64), and the tallies
// and cut-offs of Alg. 2.
//
// The samplers are independent, so they are the unit of parallelism (the
// paper spreads hyperparameters over threads for the same reason); inside a
// sampler the steps that the paper's SIMD code vectorises -- likelihoods,
// weights, ESS, moves -- run across the lanes, and the synchronising ones --
// ESS sums, resampling, the proposal covariance, the acceptance count -- are
// workgroup reductions and scans in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pps_device.hpp"
#include "pps_smc.hpp"

namespace pps {

namespace {

constexpr double TWO_POW_52 = 4503599627370496.0;
constexpr double TWO_PI = 6.283185307179586476925286766559;

__device__ __forceinline__ uint64_t wave_uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Box-Muller in FP64, both outputs: r cos(2 pi u1), r sin(2 pi u1).
__device__ __attribute__((noinline)) void box_muller_pair_f64(uint32_t w0, uint32_t w1, double &z0,
                                                              double &z1)
{
    const double u0 = uniform_f64(w0);
    const double u1 = uniform_f64(w1);
    const double r = sqrt(-2.0 * log(u0));
    double s, c;
    sincos(TWO_PI * u1, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// A double known to be equal in every lane, moved to scalar registers (frees
// the vector registers that the sampler's per-run constants would occupy).
__device__ __forceinline__ double sgpr_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ uint32_t word_of(const Words4 &w, uint32_t k)
{
    return k == 0 ? w.x : (k == 1 ? w.y : (k == 2 ? w.z : w.w));
}

// ---- workgroup reductions (fixed order: deterministic) ----------------------
// A 64-bit value moved across lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(b)), CTRL, 0xF,
                                               0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(b >> 32)), CTRL,
                                               0xF, 0xF, false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

// Sum over the 64 lanes of a wave, the same value in every lane: within each
// row of 16 lanes by DPP (quad swaps 1 and 2, then the half-row and row
// mirrors), across rows by two lane shuffles.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    v = fmax(v, __shfl_xor(v, 16, 64));
    v = fmax(v, __shfl_xor(v, 32, 64));
    return v;
}

template <int BLOCK>
__device__ __forceinline__ double wg_sum(double v, double *s_red)
{
    constexpr int NW = BLOCK / 64;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0)
        s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        tot += s_red[w];
    __syncthreads();
    return sgpr_f64(tot);
}

template <int BLOCK>
__device__ __forceinline__ void wg_sum2(double &a, double &b, double *s_red)
{
    constexpr int NW = BLOCK / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        s_red[threadIdx.x >> 6] = a;
        s_red[NW + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        ta += s_red[w];
        tb += s_red[NW + w];
    }
    __syncthreads();
    a = sgpr_f64(ta);
    b = sgpr_f64(tb);
}

template <int BLOCK>
__device__ __forceinline__ void wg_sum3(double &a, double &b, double &c, double *s_red)
{
    constexpr int NW = BLOCK / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) {
        s_red[threadIdx.x >> 6] = a;
        s_red[NW + (threadIdx.x >> 6)] = b;
        s_red[2 * NW + (threadIdx.x >> 6)] = c;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0, tc = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        ta += s_red[w];
        tb += s_red[NW + w];
        tc += s_red[2 * NW + w];
    }
    __syncthreads();
    a = sgpr_f64(ta);
    b = sgpr_f64(tb);
    c = sgpr_f64(tc);
}

template <int BLOCK>
__device__ __forceinline__ double wg_max(double v, double *s_red)
{
    constexpr int NW = BLOCK / 64;
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0)
        s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = s_red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
        m = fmax(m, s_red[w]);
    __syncthreads();
    return sgpr_f64(m);
}

template <int BLOCK>
__device__ __forceinline__ int wg_count(bool pred, unsigned *s_cnt)
{
    constexpr int NW = BLOCK / 64;
    const unsigned c = static_cast<unsigned>(__popcll(__ballot(pred)));
    if ((threadIdx.x & 63) == 0)
        s_cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        tot += static_cast<int>(s_cnt[w]);
    __syncthreads();
    return tot;
}

// Inclusive prefix sums of 64-bit integers over the workgroup, into s_cum.
template <int BLOCK>
__device__ __forceinline__ void wg_scan_u64(uint64_t x, unsigned long long *s_cum,
                                            unsigned long long *s_wave)
{
    constexpr int NW = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t lo = __shfl_up(static_cast<uint32_t>(x), off, 64);
        const uint32_t hi = __shfl_up(static_cast<uint32_t>(x >> 32), off, 64);
        if (lane >= off)
            x += (static_cast<uint64_t>(hi) << 32) | lo;
    }
    if (lane == 63)
        s_wave[wave] = x;
    __syncthreads();
    uint64_t base = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        if (w < wave)
            base += s_wave[w];
    s_cum[threadIdx.x] = x + base;
    __syncthreads();
}

// ---- the model ---------------------------------------------------------------
// Groups of the current data set in LDS (the same for every lane): trials n,
// deaths k, dose x; lcoef = sum_i log C(n_i, k_i).
struct GroupsLds {
    double n[PPS_BIO_MAX_GROUPS], k[PPS_BIO_MAX_GROUPS], x[PPS_BIO_MAX_GROUPS];
};

// log L(theta; D) (Eq. bioassay): sum_i log C(n_i, y_i) + sum_i [-y_i s_i +
// (n_i - y_i)(eta_i - s_i)], s_i = log(1 + e^eta_i), eta_i = b0 + b1 x_i.
__device__ __forceinline__ double bio_loglik(const GroupsLds &g, int m, double lcoef, double b0,
                                             double b1)
{
    double ll = lcoef;
#pragma unroll 1
    for (int i = 0; i < m; ++i) {
        const double eta = b0 + b1 * g.x[i];
        const double sp = eta > 0.0 ? eta + log1p(exp(-eta)) : log1p(exp(eta));
        ll += -g.k[i] * sp + (g.n[i] - g.k[i]) * (eta - sp);
    }
    return ll;
}

__device__ __forceinline__ double bio_logprior(double l0, double l1, double b0, double b1)
{
    const double a = b0 / l0, c = b1 / l1;
    return -0.5 * (a * a + c * c) - log(TWO_PI * l0 * l1);
}

}  // namespace

// ===========================================================================
// Data sets D ~ p(D | lambda): theta from Box-Muller on words (0, 1) of block
// 0; group i counts its trials whose uniform (words of blocks 1, 2, ... in
// order) is below p_i = 1 / (1 + exp(b0 + b1 x_i)).  One thread per data set:
// the base sets D_0^(i) first, then D_k^(i) for every k.
// ===========================================================================
__global__ void k_bio_data(BioDesign b, const double *__restrict__ lam, int n_lambda,
                           uint64_t n_data, uint64_t seed, int32_t *__restrict__ y0,
                           int32_t *__restrict__ yk, double *__restrict__ lcoef)
{
    __shared__ double s_dose[PPS_BIO_MAX_GROUPS];
    __shared__ int s_trials[PPS_BIO_MAX_GROUPS];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < PPS_BIO_MAX_GROUPS; ++j) {
            s_dose[j] = b.dose[j];
            s_trials[j] = b.n_trials[j];
        }
    }
    __syncthreads();
    const StreamKey key = make_key(seed);
    const uint64_t total = n_data * (1 + static_cast<uint64_t>(n_lambda));
    const int m = b.n_groups;
    for (uint64_t q = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; q < total;
         q += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        uint64_t id;
        uint32_t purpose;
        double l0, l1;
        int32_t *out;
        if (q < n_data) {
            id = q;
            purpose = SMC_P_DATA_BASE;
            l0 = lam[0];
            l1 = lam[1];
            out = y0 + q * m;
        } else {
            id = q - n_data;
            const uint64_t k = id / n_data;
            purpose = SMC_P_DATA_K;
            l0 = lam[2 * k];
            l1 = lam[2 * k + 1];
            out = yk + id * m;
        }
        const Words4 w0 = stream_block(key, id, 0, purpose);
        double z0, z1;
        box_muller_pair_f64(w0.x, w0.y, z0, z1);
        const double b0 = l0 * z0, b1 = l1 * z1;
        uint32_t k = 0;
        Words4 cur = w0;
        double lc = 0.0;
        for (int i = 0; i < m; ++i) {
            const double p = 1.0 / (1.0 + exp(b0 + b1 * s_dose[i]));
            int32_t count = 0;
            for (int r = 0; r < s_trials[i]; ++r, ++k) {
                if ((k & 3) == 0)
                    cur = stream_block(key, id, 1 + (k >> 2), purpose);
                if (uniform_f64(word_of(cur, k & 3)) < p)
                    ++count;
            }
            out[i] = count;
            const double nn = s_trials[i], kk = count;
            lc += lgamma(nn + 1.0) - lgamma(kk + 1.0) - lgamma(nn - kk + 1.0);
        }
        lcoef[q] = lc;
    }
}

// ===========================================================================
// The adaptive SMC sampler (Alg. 3), one run per workgroup, particle j on
// lane j.  Persistent: workgroups take runs from an atomic counter.  Every
// loop that lane 0 runs alone is avoided at the end of a run (the distance
// between two tiles' barriers must hold no divergent loop), and a run ends
// with a barrier.
// ===========================================================================
// Four waves per SIMD (at most 128 VGPRs; a few loop-invariant values spill)
// run ~25 % faster than the two that the unconstrained allocation leaves.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_smc(
    BioDesign b, SmcParams P, uint64_t seed, SmcRuns R)
{
    constexpr int NW = BLOCK / 64;
    __shared__ double s_b0[BLOCK], s_b1[BLOCK], s_ll[BLOCK];
    __shared__ unsigned long long s_cum[BLOCK];
    __shared__ double s_red[3 * NW];
    __shared__ unsigned long long s_wave[NW];
    __shared__ unsigned s_cnt[NW];
    __shared__ unsigned long long s_tile;
    __shared__ GroupsLds s_g;
    const int tid = threadIdx.x;
    const int np = P.n_particles;
    const bool live = tid < np;
    const StreamKey key = make_key(seed);
    const double half = 0.5 * np;
    for (;;) {
        if (tid == 0)
            s_tile = atomicAdd(R.next_run, 1ull);
        __syncthreads();
        const uint64_t r = wave_uniform_u64(s_tile);
        __syncthreads();
        if (r >= R.n_runs)
            break;
        const int32_t *y;
        const double *lam, *lc;
        uint64_t run;
        double *out;
        if (R.mode == 0) {
            y = R.y + r * b.n_groups;
            lc = R.lcoef + r;
            lam = R.lam + 2 * r;
            run = R.first_run + r;
            out = R.out0 + r;
        } else {
            const uint64_t ki = r >> 1;
            const uint64_t k = ki / R.n_data, i = ki % R.n_data;
            const bool base = (r & 1) == 0;
            y = base ? R.y + i * b.n_groups : R.yk + ki * b.n_groups;
            lc = base ? R.lcoef + i : R.lcoef + R.n_data + ki;
            lam = R.lam + 2 * k;
            run = r;
            out = (base ? R.out0 : R.outk) + ki;
        }
        const double l0 = sgpr_f64(lam[0]), l1 = sgpr_f64(lam[1]);
        const int m = b.n_groups;
        if (tid < m) {
            // static indices into the by-value design (a lane index would
            // place the argument in scratch memory)
            double nn = 0.0, xx = 0.0;
#pragma unroll
            for (int j = 0; j < PPS_BIO_MAX_GROUPS; ++j) {
                if (j == tid) {
                    nn = static_cast<double>(b.n_trials[j]);
                    xx = b.dose[j];
                }
            }
            s_g.n[tid] = nn;
            s_g.k[tid] = static_cast<double>(y[tid]);
            s_g.x[tid] = xx;
        }
        __syncthreads();
        const double lcoef = sgpr_f64(*lc);
        // initial particles from the prior
        double b0 = 0.0, b1 = 0.0, ll = -INFINITY;
        if (live) {
            const Words4 w = stream_block(key, run, 0, SMC_P_INIT + static_cast<uint32_t>(tid));
            double z0, z1;
            box_muller_pair_f64(w.x, w.y, z0, z1);
            b0 = l0 * z0;
            b1 = l1 * z1;
            ll = bio_loglik(s_g, m, lcoef, b0, b1);
        }
        double t = 0.0, log_z = 0.0;
        for (int n = 1;; ++n) {
            const double lmax = wg_max<BLOCK>(ll, s_red);
            const double rest = 1.0 - t;
            // the tempering increment: ESS of exp(delta (l - l_max)) = N_p / 2
            double s = live ? exp(rest * (ll - lmax)) : 0.0, s2 = s * s;
            wg_sum2<BLOCK>(s, s2, s_red);
            double delta = rest;
            if (!(n >= P.max_steps || s * s / s2 >= half)) {
                double lo = 0.0, hi = rest;
                for (int it = 0; it < P.bisect_iters; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    double a = live ? exp(mid * (ll - lmax)) : 0.0, a2 = a * a;
                    wg_sum2<BLOCK>(a, a2, s_red);
                    if (a * a / a2 >= half)
                        lo = mid;
                    else
                        hi = mid;
                }
                delta = lo;
            }
            const double w = live ? exp(delta * (ll - lmax)) : 0.0;
            const double sum_w = wg_sum<BLOCK>(w, s_red);
            log_z = sgpr_f64(log_z + (delta * lmax + log(sum_w / np)));
            if (delta == rest)
                break;  // t = 1: the evidence is complete
            t = sgpr_f64(t + delta);
            // multinomial resampling by inversion of fixed-point weights
            const uint64_t q = live ? static_cast<uint64_t>(floor(w * TWO_POW_52)) : 0ull;
            s_b0[tid] = b0;
            s_b1[tid] = b1;
            s_ll[tid] = ll;
            wg_scan_u64<BLOCK>(q, s_cum, s_wave);
            const uint64_t total = s_cum[np - 1];
            if (live) {
                const Words4 wr =
                    stream_block(key, run, static_cast<uint32_t>(n), SMC_P_RESAMPLE + static_cast<uint32_t>(tid));
                const uint64_t r64 = (static_cast<uint64_t>(wr.y) << 32) | wr.x;
                const uint64_t u = __umul64hi(r64, total);
                int lo = 0, hi = np - 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (s_cum[mid] > u)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                b0 = s_b0[lo];
                b1 = s_b1[lo];
                ll = s_ll[lo];
            }
            __syncthreads();
            // proposal N(0, h^2 Sigma_hat): sample covariance of the particles
            double m0 = live ? b0 : 0.0, m1 = live ? b1 : 0.0;
            wg_sum2<BLOCK>(m0, m1, s_red);
            m0 /= np;
            m1 /= np;
            const double d0 = b0 - m0, d1 = b1 - m1;
            double c00 = live ? d0 * d0 : 0.0, c01 = live ? d0 * d1 : 0.0, c11 = live ? d1 * d1 : 0.0;
            wg_sum3<BLOCK>(c00, c01, c11, s_red);
            c00 /= (np - 1);
            c01 /= (np - 1);
            c11 /= (np - 1);
            const double h2 = P.h * P.h;
            const double f11 = sgpr_f64(c00 > 0.0 ? sqrt(h2 * c00) : 0.0);
            const double f21 = sgpr_f64(c00 > 0.0 ? h2 * c01 / f11 : 0.0);
            const double r22 = h2 * c11 - f21 * f21;
            const double f22 = sgpr_f64(r22 > 0.0 ? sqrt(r22) : 0.0);
            // Metropolis-Hastings moves targeting L^t pi(theta | lambda)
            int moves = 1;
            for (int mv = 0; mv < moves; ++mv) {
                bool acc = false;
                if (live) {
                    const Words4 wm = stream_block(
                        key, run, static_cast<uint32_t>(n * SMC_BLOCKS_PER_STEP + mv),
                        SMC_P_MCMC + static_cast<uint32_t>(tid));
                    double z0, z1;
                    box_muller_pair_f64(wm.x, wm.y, z0, z1);
                    const double p0 = b0 + f11 * z0;
                    const double p1 = b1 + f21 * z0 + f22 * z1;
                    const double pll = bio_loglik(s_g, m, lcoef, p0, p1);
                    const double log_alpha = t * (pll - ll) + bio_logprior(l0, l1, p0, p1) -
                                             bio_logprior(l0, l1, b0, b1);
                    if (log(uniform_f64(wm.z)) < log_alpha) {
                        b0 = p0;
                        b1 = p1;
                        ll = pll;
                        acc = true;
                    }
                }
                if (mv == 0) {
                    const int accepted = wg_count<BLOCK>(acc, s_cnt);
                    if (accepted <= 0) {
                        moves = P.max_mcmc;
                    } else if (accepted >= np) {
                        moves = 1;
                    } else {
                        const double rn = ceil(log(P.c) / log(1.0 - static_cast<double>(accepted) / np));
                        moves = rn < 1.0 ? 1 : (rn > P.max_mcmc ? P.max_mcmc : static_cast<int>(rn));
                    }
                }
            }
        }
        if (tid == 0)
            *out = log_z;
        __syncthreads();
    }
}

// ===========================================================================
// Alg. 2 tallies: counts c_i = #{j : log pi_k^j <= log pi_0^i} (p = c / N),
// then gamma_k = the q-th smallest p of row k: the smallest c_i with
// #{j : c_j <= c_i} >= q.
// ===========================================================================
__global__ void k_wip_counts(const double *__restrict__ z0, const double *__restrict__ zk,
                             int n_lambda, uint64_t n_data, uint32_t *__restrict__ counts,
                             double *__restrict__ pvals)
{
    const uint64_t total = static_cast<uint64_t>(n_lambda) * n_data;
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t k = e / n_data;
        const double v = z0[e];
        const double *row = zk + k * n_data;
        uint32_t c = 0;
        for (uint64_t j = 0; j < n_data; ++j)
            c += row[j] <= v ? 1u : 0u;
        counts[e] = c;
        if (pvals)
            pvals[e] = static_cast<double>(c) / static_cast<double>(n_data);
    }
}

__global__ __launch_bounds__(256) void k_wip_gamma(const uint32_t *__restrict__ counts, int n_lambda,
                                                   uint64_t n_data, uint64_t q,
                                                   double *__restrict__ gamma)
{
    __shared__ uint32_t s_min[4];
    for (int k = blockIdx.x; k < n_lambda; k += gridDim.x) {
        const uint32_t *row = counts + static_cast<uint64_t>(k) * n_data;
        uint32_t best = 0xFFFFFFFFu;
        for (uint64_t i = threadIdx.x; i < n_data; i += blockDim.x) {
            const uint32_t ci = row[i];
            uint64_t rank = 0;
            for (uint64_t j = 0; j < n_data; ++j)
                rank += row[j] <= ci ? 1u : 0u;
            if (rank >= q && ci < best)
                best = ci;
        }
        for (int off = 32; off > 0; off >>= 1)
            best = min(best, static_cast<uint32_t>(__shfl_xor(static_cast<int>(best), off, 64)));
        if ((threadIdx.x & 63) == 0)
            s_min[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t m = min(min(s_min[0], s_min[1]), min(s_min[2], s_min[3]));
            gamma[k] = static_cast<double>(m) / static_cast<double>(n_data);
        }
        __syncthreads();
    }
}

// ===========================================================================
// Host launchers.
// ===========================================================================
int smc_block_for(int n_particles)
{
    return n_particles <= 256 ? 256 : (n_particles <= 512 ? 512 : 1024);
}

hipError_t smc_occupancy(int block, int *blocks_per_cu)
{
    switch (block) {
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_smc<256>, 256, 0);
    case 512: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_smc<512>, 512, 0);
    case 1024:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_smc<1024>, 1024, 0);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bio_data(const BioDesign &b, const double *lam, int n_lambda, uint64_t n_data,
                           uint64_t seed, int32_t *y0, int32_t *yk, double *lcoef, hipStream_t s)
{
    const uint64_t total = n_data * (1 + static_cast<uint64_t>(n_lambda));
    const unsigned grid = static_cast<unsigned>(std::min<uint64_t>((total + 255) / 256, 4096));
    hipLaunchKernelGGL(k_bio_data, dim3(grid), dim3(256), 0, s, b, lam, n_lambda, n_data, seed, y0,
                       yk, lcoef);
    return hipGetLastError();
}

hipError_t launch_smc(const BioDesign &b, const SmcParams &p, uint64_t seed, const SmcRuns &runs,
                      unsigned grid, hipStream_t s)
{
    switch (smc_block_for(p.n_particles)) {
    case 256: hipLaunchKernelGGL(k_smc<256>, dim3(grid), dim3(256), 0, s, b, p, seed, runs); break;
    case 512: hipLaunchKernelGGL(k_smc<512>, dim3(grid), dim3(512), 0, s, b, p, seed, runs); break;
    default: hipLaunchKernelGGL(k_smc<1024>, dim3(grid), dim3(1024), 0, s, b, p, seed, runs); break;
    }
    return hipGetLastError();
}

hipError_t launch_wip_tally(const double *z0, const double *zk, int n_lambda, uint64_t n_data,
                            uint64_t q, uint32_t *counts, double *pvals, double *gamma,
                            hipStream_t s)
{
    const uint64_t total = static_cast<uint64_t>(n_lambda) * n_data;
    const unsigned grid = static_cast<unsigned>(std::min<uint64_t>((total + 255) / 256, 8192));
    hipLaunchKernelGGL(k_wip_counts, dim3(grid), dim3(256), 0, s, z0, zk, n_lambda, n_data, counts,
                       pvals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_wip_gamma, dim3(std::min(n_lambda, 4096)), dim3(256), 0, s, counts,
                       n_lambda, n_data, q, gamma);
    return hipGetLastError();
}

}  // namespace pps
