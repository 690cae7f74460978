// BEGE log-likelihood on gfx950 (Sec. 4.2: Eqs. BEGE, shape, BEGE_LL,
// CDF_BEGE, BEGE_LL_approx, incompGamma), FP64.
//
// The paper vectorises the incomplete gamma function across the quadrature
// nodes of one transition density.  Here the unit of parallelism is the
// transition density itself: the shapes (p_{t-1}, n_{t-1}) of every
// (parameter vector, t) are known once the shape recursion has run over the
// data, so the T densities of a parameter vector are independent and go one
// per lane, 64 consecutive t of one vector per wave (neighbouring t have
// similar shapes, so the lanes' series lengths stay close).  Kernels:
//   k_bege_shapes   one wave per vector: the recursion of Eq. shape as a scan
//                   over chunks of 64 steps, and a cost class per chunk from
//                   its largest shape;
//   k_bege_order    one workgroup: the chunks in decreasing cost class;
//   k_bege_density  one lane per (vector, t): log f(u_t | p_{t-1}, n_{t-1}),
//                   chunks taken in that order so that the long waves (large
//                   shapes need long series) start first and the short ones
//                   fill in behind them;
//   k_bege_sum      one workgroup per vector: log L, summed in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pps_bege.hpp"

namespace pps {

namespace {

constexpr int DENSITY_BLOCK = 64;
constexpr int SUM_BLOCK = 256;
constexpr int SHAPES_BLOCK = 64;
constexpr int ORDER_BLOCK = 1024;
constexpr int N_COST_CLASSES = 64;

// Regularised incomplete gamma: truncation and iteration cap.
constexpr double IG_EPS = 1.1102230246251565e-16;  // 2^-53
constexpr int IG_MAXIT = 100000;

// theta = (p0, s_p, rho_p, phi_p+, phi_p-, n0, s_n, rho_n, phi_n+, phi_n-, mu)
enum { P0, SP, RP, PPOS, PNEG, N0, SN, RN, NPOS, NNEG, MU };

// Operation counting (the COUNT instantiation, for measurement only): FP64
// operations per lane as the method states them, an FMA counting 2 (as the
// FP64 peak counts it), a division 1, and exp, log, lgamma and sqrt 1 each
// (one operation of the method, whatever their instruction cost on the
// device: that shows in the instruction counters, not here).
constexpr double OPS_EXP = 1.0, OPS_LOG = 1.0, OPS_LGAMMA = 1.0;
constexpr double OPS_SERIES_IT = 5.0, OPS_SERIES_CHECK = 1.0, OPS_CF_IT = 10.0, OPS_CF_CHECK = 4.0;
constexpr double OPS_IGAM_FIXED = OPS_LOG + OPS_EXP + 6.0;
constexpr double OPS_TAYLOR = 62.0 + OPS_LOG + OPS_EXP;

template <bool COUNT>
struct OpCount {
    double v = 0.0;
    __device__ __forceinline__ void add(double k)
    {
        if constexpr (COUNT)
            v += k;
    }
};

// P(a, x) of Eq. incompGamma for x > 0, given ln Gamma(a), without a
// division inside either loop (an FP64 division costs a dozen instructions on
// this GPU, a multiply one):
//   x < a + 1: e^-x x^a / Gamma(a + 1) times S = sum_m x^m / prod_{i<=m}(a+i).
//     S is carried as N / D with D = prod (a+i), N = D S, X = x^m:
//     N <- N (a+k) + X; the series is cut once a term is below 2^-53 of the
//     sum, i.e. X < 2^-53 N;
//   x >= a + 1: 1 - e^-x x^a / Gamma(a) / K with Legendre's continued fraction
//     K = b_0 + a_1 / (b_1 + a_2 / (b_2 + ...)), b_i = x + 2i + 1 - a,
//     a_i = -i (i - a), by the convergents A_i / B_i of the three-term
//     recurrences (A, B)_i = b_i (A, B)_{i-1} + a_i (A, B)_{i-2}; it stops
//     once successive values of 1/K agree to 2^-53, i.e.
//     |B_i A_{i-1} - A_i B_{i-1}| < 2^-53 |A_i B_{i-1}|.
// Both loops run in blocks (8 series terms, 4 fraction steps) and test
// convergence and scale at the end of a block: a block adds at most a few
// terms past the cut, each below 2^-53 of the result.  One term multiplies
// the values by at most a + k (series) or x + a + 4k (fraction), so a block
// grows them by less than 2^400 while a, x < 2^40 (shapes within the priors
// stay far below); larger arguments take blocks of one term, safe up to
// 2^400.  N, D, X (and A, B) are scaled by 2^-600 together when they pass
// 2^600: exact, and only their ratios are used.
template <int BLK>
__device__ __forceinline__ double igam_series(double a, double x, int &k)
{
    double n = 1.0, d = 1.0, xm = 1.0, ak = a;
    k = 0;
    do {
#pragma unroll
        for (int u = 0; u < BLK; ++u) {
            ak += 1.0;
            xm *= x;
            n = fma(n, ak, xm);
            d *= ak;
        }
        k += BLK;
        if (xm < n * IG_EPS)
            break;
        if (d > 0x1p600) {
            n *= 0x1p-600;
            d *= 0x1p-600;
            xm *= 0x1p-600;
        }
    } while (k < IG_MAXIT);
    return n / (a * d);
}

// 1/K; steps in pairs so that (A1, B1) is always the latest convergent and
// (A0, B0) the one before.
template <int BLK>
__device__ __forceinline__ double igam_fraction(double a, double x, int &i)
{
    double A0 = 1.0, A1 = x + 1.0 - a, B0 = 0.0, B1 = 1.0, bi = A1, di = 0.0;
    i = 0;
    do {
#pragma unroll
        for (int u = 0; u < BLK; ++u) {
            di += 1.0;
            bi += 2.0;
            const double ai = -di * (di - a);
            if (u % 2 == 0) {
                A0 = fma(bi, A1, ai * A0);
                B0 = fma(bi, B1, ai * B0);
            } else {
                A1 = fma(bi, A0, ai * A1);
                B1 = fma(bi, B0, ai * B1);
            }
        }
        if (BLK % 2 == 1) {
            // odd block: bring the latest convergent back to (A1, B1)
            const double ta = A0, tb = B0;
            A0 = A1;
            B0 = B1;
            A1 = ta;
            B1 = tb;
        }
        i += BLK;
        const double cross = A1 * B0;
        const double diff = fma(B1, A0, -cross);
        if (fabs(diff) < IG_EPS * fabs(cross))
            break;
        if (fabs(A1) > 0x1p600) {
            A0 *= 0x1p-600;
            A1 *= 0x1p-600;
            B0 *= 0x1p-600;
            B1 *= 0x1p-600;
        }
    } while (i < IG_MAXIT);
    return B1 / A1;
}

constexpr int SERIES_BLOCK = 8;
constexpr int CF_BLOCK = 4;

template <bool COUNT>
__device__ __attribute__((noinline)) double igam_p(double a, double x, double lga, OpCount<COUNT> &ops)
{
    if (!(x > 0.0))
        return 0.0;
    const double e = a * log(x) - x - lga;
    const bool blocked = a < 0x1p40 && x < 0x1p40;
    int it;
    if (x < a + 1.0) {
        const double s = blocked ? igam_series<SERIES_BLOCK>(a, x, it) : igam_series<1>(a, x, it);
        ops.add(OPS_IGAM_FIXED + OPS_SERIES_IT * it + OPS_SERIES_CHECK * (it / (blocked ? SERIES_BLOCK : 1)));
        return exp(e) * s;
    }
    const double f = blocked ? igam_fraction<CF_BLOCK>(a, x, it) : igam_fraction<1>(a, x, it);
    ops.add(OPS_IGAM_FIXED + OPS_CF_IT * it + OPS_CF_CHECK * (it / (blocked ? CF_BLOCK : 1)));
    return 1.0 - exp(e) * f;
}

// Q(a, x) = 1 - P(a, x) for x >= a + 1, straight from the continued fraction
// (e^-x x^a / Gamma(a) / K): in the upper tail Q keeps its relative accuracy,
// where 1 - P would be within rounding of 0.
template <bool COUNT>
__device__ __attribute__((noinline)) double igam_q_upper(double a, double x, double lga, OpCount<COUNT> &ops)
{
    const double e = a * log(x) - x - lga;
    const bool blocked = a < 0x1p40 && x < 0x1p40;
    int it;
    const double f = blocked ? igam_fraction<CF_BLOCK>(a, x, it) : igam_fraction<1>(a, x, it);
    ops.add(OPS_IGAM_FIXED + OPS_CF_IT * it + OPS_CF_CHECK * (it / (blocked ? CF_BLOCK : 1)));
    return exp(e) * f;
}

// 1/x to FP64 accuracy from the hardware reciprocal and two Newton steps
// (each step squares the relative error), where a correctly rounded IEEE
// division is not needed: a few instructions instead of a dozen.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// The Gamma(a, 1) density integrated over one node interval, relative to its
// value at one end, by the Taylor series of the density about that end (the
// distribution function of Eq. BEGE_LL_approx needs only the increments of
// P(a, .) between consecutive nodes, and the integral of its density over the
// interval is such an increment).  About the end X where the density is the
// smaller one (the left end x if x < a - 1, where the density rises, else the
// right end x + dx), the density at distance t into the interval is its value
// at X times
//   k(t) = (1 - s t / X)^(a - 1) e^(s t),   s = -1 about the left end, +1 about the right,
// a function that grows into the interval, so the series' terms keep one sign
// up to the small curvature term.  From (X - s t) k' = s (X - a + 1 - s t) k,
// the coefficients scaled by dx^m, e_m = k_m dx^m, follow
//   e_0 = 1,  e_{m+1} = ((B + s m) beta e_m - beta dx e_{m-1}) / (m + 1),
//   B = s (X - a + 1),  beta = dx / X,
// and the interval's integral is dx sum_m e_m / (m + 1), the density at the
// other end the value at X times sum_m e_m.  The series converges for beta < 1
// (the singularity of k at t = s X); the caller takes it where beta <= 1/2 and
// the log-density changes by little over the interval, and it stops once two
// consecutive terms are below 2^-54 of the integral, or gives up (ok = false)
// after TAYLOR_BLOCKS blocks of four terms.
constexpr int TAYLOR_BLOCKS = 12;
constexpr double TAYLOR_L1 = 8.0;    // bound on |d ln g / dx| dx over the interval
constexpr double TAYLOR_CURV = 4.0;  // bound on |a - 1| beta^2 (the curvature term)
constexpr double OPS_TAYLOR_TERM = 8.0, OPS_TAYLOR_CHECK = 3.0;

struct TaylorSum {
    double I;  // sum_m e_m / (m + 1)
    double H;  // sum_m e_m
    bool ok;
};

template <bool COUNT>
__device__ __attribute__((noinline)) TaylorSum gamma_taylor(double B, double beta, double dx, double s,
                                                            OpCount<COUNT> &ops)
{
    const double gam = beta * dx;
    const double step = s * beta;
    double em1 = 0.0, e = 1.0, t = B * beta;
    TaylorSum r;
    r.I = 1.0;
    r.H = 1.0;
    r.ok = false;
    int blocks = 0;
#pragma unroll
    for (int blk = 0; blk < TAYLOR_BLOCKS; ++blk) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int m = 4 * blk + u;  // e_{m+1} from e_m and e_{m-1}
            const double en = fma(t, e, -gam * em1) * (1.0 / (m + 1));
            t += step;
            em1 = e;
            e = en;
            r.I = fma(e, 1.0 / (m + 2), r.I);
            r.H += e;
        }
        blocks = blk + 1;
        if (fabs(e) + fabs(em1) <= 0x1p-54 * r.I) {
            r.ok = true;
            break;
        }
    }
    ops.add(4.0 + blocks * (4.0 * OPS_TAYLOR_TERM + OPS_TAYLOR_CHECK));
    return r;
}

// Cost class of a chunk from the largest shape p among its valid steps: the
// series of P(p, x) near x = p need about sqrt(p) terms, so the class is
// 2 log2(max p) + 16 clamped to [1, 63] (quarter octaves of sqrt p); a chunk
// with no valid step is class 0.
__device__ __forceinline__ int cost_class(double pmax)
{
    if (!(pmax > 0.0))
        return 0;
    const int c = static_cast<int>(2.0 * log2(pmax)) + 16;
    return c < 1 ? 1 : (c > N_COST_CLASSES - 1 ? N_COST_CLASSES - 1 : c);
}

// The recursion p_t = rho p_{t-1} + c_t, c_t = p0 + phi^{+/-} u_t^2 / (2 s^2),
// is affine with a constant multiplier, so a wave scans it 64 steps at a
// time: lane j of a chunk starting at step t_c holds c_{t_c + j}, an
// inclusive scan v_j = sum_{s <= j} rho^{j-s} c_{t_c + s} takes six shuffle
// steps, and the shape meeting step t_c + j is rho^j P + v_{j-1}, P the
// shape carried into the chunk (p_{t_c - 1}).  One wave per vector; the
// shapes leave as contiguous rows.  (The sums are associated differently
// from the step-by-step recursion: rounding-level differences.)
__device__ __forceinline__ double shfl_up_f64(double v, int d)
{
    return __shfl_up(v, d, 64);
}

__global__ __launch_bounds__(SHAPES_BLOCK) void k_bege_shapes(BegeBatch b)
{
    static_assert(SHAPES_BLOCK == 64 && DENSITY_BLOCK == 64, "one wave per vector, chunks of 64");
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const double *th = b.theta + static_cast<size_t>(k) * BEGE_NPAR;
    const double p0 = th[P0], sp = th[SP], rp = th[RP], ppos = th[PPOS], pneg = th[PNEG];
    const double n0 = th[N0], sn = th[SN], rn = th[RN], npos = th[NPOS], nneg = th[NNEG];
    const double mu = th[MU];
    const double cp = 0.5 / (sp * sp), cn = 0.5 / (sn * sn);
    const bool scales_ok = sp > 0.0 && sn > 0.0;
    // rho^j for this lane and rho^(2^i) for the scan (squarings)
    double rpow[6], npow[6];
    rpow[0] = rp;
    npow[0] = rn;
#pragma unroll
    for (int i = 1; i < 6; ++i) {
        rpow[i] = rpow[i - 1] * rpow[i - 1];
        npow[i] = npow[i - 1] * npow[i - 1];
    }
    double rj = 1.0, nj = 1.0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        if (lane & (1 << i)) {
            rj *= rpow[i];
            nj *= npow[i];
        }
    const double r64 = rpow[5] * rpow[5], n64 = npow[5] * npow[5];
    double P = p0, N = n0;  // shapes carried into the chunk
    double *outp = b.shape_p + static_cast<size_t>(k) * b.T;
    double *outn = b.shape_n + static_cast<size_t>(k) * b.T;
    for (int c = 0; c < b.chunks; ++c) {
        const int t = c * DENSITY_BLOCK + lane + 1;
        const bool in = t <= b.T;
        const double u = in ? b.r[t] - mu : 0.0;
        const double u2 = u * u;
        const bool pos = u >= 0.0;
        double vp = in ? p0 + (pos ? ppos : pneg) * u2 * cp : 0.0;
        double vn = in ? n0 + (pos ? npos : nneg) * u2 * cn : 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const int d = 1 << i;
            const double op = shfl_up_f64(vp, d), on = shfl_up_f64(vn, d);
            if (lane >= d) {
                vp = fma(rpow[i], op, vp);
                vn = fma(npow[i], on, vn);
            }
        }
        // exclusive value v_{j-1} and the shape meeting step t
        const double ep = shfl_up_f64(vp, 1), en = shfl_up_f64(vn, 1);
        const double shp = fma(rj, P, lane > 0 ? ep : 0.0);
        const double shn = fma(nj, N, lane > 0 ? en : 0.0);
        if (in) {
            outp[t - 1] = shp;
            outn[t - 1] = shn;
        }
        // carry: p at the chunk's last step = rho^64 P + v_63
        const double last_p = __shfl(vp, 63, 64), last_n = __shfl(vn, 63, 64);
        P = fma(r64, P, last_p);
        N = fma(n64, N, last_n);
        // cost class from the largest valid shape of the chunk
        double pm = (in && scales_ok && shp > 0.0 && shn > 0.0) ? shp : 0.0;
#pragma unroll
        for (int m = 32; m > 0; m >>= 1)
            pm = fmax(pm, __shfl_xor(pm, m, 64));
        if (lane == 0)
            b.chunk_class[static_cast<size_t>(k) * b.chunks + c] = cost_class(pm);
    }
}

// Counting sort of the chunks by decreasing cost class (one workgroup; the
// order within a class is immaterial: every chunk writes its own outputs).
__global__ __launch_bounds__(ORDER_BLOCK) void k_bege_order(BegeBatch b)
{
    __shared__ unsigned hist[N_COST_CLASSES];
    __shared__ unsigned start[N_COST_CLASSES];
    const uint32_t n = static_cast<uint32_t>(b.n_theta) * static_cast<uint32_t>(b.chunks);
    if (threadIdx.x < N_COST_CLASSES)
        hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += ORDER_BLOCK)
        atomicAdd(&hist[b.chunk_class[i]], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned acc = 0;
        for (int c = N_COST_CLASSES - 1; c >= 0; --c) {
            start[c] = acc;
            acc += hist[c];
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += ORDER_BLOCK)
        b.chunk_order[atomicAdd(&start[b.chunk_class[i]], 1u)] = static_cast<int32_t>(i);
}

// Integral of the Gamma(n, 1) density over [y_m - d/2, y_m + d/2] by its
// Taylor series about the midpoint,
//   d g(y_m) [1 + B_2 d^2/24 + B_4 d^4/1920 + B_6 d^6/322560],
// with g^(k) / g = B_k(L_1, ..., L_k) (complete Bell polynomials) of the
// derivatives of L = ln g: L_1 = c/y - 1, L_k = (-1)^(k-1) (k-1)! c / y^k
// (k >= 2), c = n - 1.  With z = d (|L_1| + (1 + sqrt|c|)/y) <= 0.03 every
// omitted term is below 2^-52 of the sum.  lg = ln Gamma(n).
__device__ __forceinline__ double gamma_mass_taylor(double c, double ym, double v, double L1, double d,
                                                    double lg)
{
    const double cv = c * v;
    const double L2 = -cv * v;
    const double L3 = -2.0 * L2 * v;
    const double L4 = -3.0 * L3 * v;
    const double L5 = -4.0 * L4 * v;
    const double L6 = -5.0 * L5 * v;
    const double a2 = L1 * L1;
    const double B2 = a2 + L2;
    const double B4 = a2 * (a2 + 6.0 * L2) + 4.0 * L1 * L3 + 3.0 * L2 * L2 + L4;
    const double B6 = a2 * (a2 * (a2 + 15.0 * L2) + 20.0 * L1 * L3 + 45.0 * L2 * L2 + 15.0 * L4) +
                      L2 * (15.0 * L2 * L2 + 60.0 * L1 * L3 + 15.0 * L4) + 10.0 * L3 * L3 + 6.0 * L1 * L5 +
                      L6;
    const double d2 = d * d;
    const double g = exp(c * log(ym) - ym - lg);
    return d * g * (1.0 + d2 * (B2 * (1.0 / 24.0) + d2 * (B4 * (1.0 / 1920.0) + d2 * (B6 * (1.0 / 322560.0)))));
}

// Gamma(n, 1) mass of [ylo, yhi] for yhi <= 2 by the termwise integral of
// y^(n-1) e^-y = sum_k (-1)^k y^(n-1+k) / k!:
//   mass = yhi^n / Gamma(n) sum_k (-yhi)^k / (k! (n + k)) (1 - rho^(n+k)),
// rho = ylo / yhi (0 when ylo <= 0), with
//   1 - rho^(n+k) = A + (1 - A)(1 - rho) G_k,  A = 1 - rho^n = -expm1(n log1p(-(1 - rho))),
//   1 - rho = (yhi - ylo) / yhi,  G_k = 1 + rho + ... + rho^(k-1),
// so every factor is formed without cancellation and a short interval keeps
// its relative accuracy where P(n, yhi) - P(n, ylo) would not (both near 1
// for a small shape).  The alternating sum loses at most a factor e^(2 yhi)
// <= e^4 of relative accuracy.
template <bool COUNT>
__device__ __attribute__((noinline)) double gamma_mass_low(double n, double ylo, double yhi, double lgn,
                                                           OpCount<COUNT> &ops)
{
    const double lead = exp(n * log(yhi) - lgn);
    double A = 1.0, om = 1.0, rho = 0.0;
    if (ylo > 0.0) {
        om = (yhi - ylo) / yhi;
        rho = ylo / yhi;
        A = -expm1(n * log1p(-om));
    }
    const double rn = 1.0 - A;  // rho^n
    const double rom = rn * om;
    double G = 0.0, term = 1.0, sum = 0.0;
    int k = 0;
    for (; k < 200; ++k) {
        const double t = term * fma(rom, G, A) / (n + static_cast<double>(k));
        sum += t;
        if (k > 0 && fabs(t) < IG_EPS * fabs(sum))
            break;
        term *= -yhi / static_cast<double>(k + 1);
        G = fma(rho, G, 1.0);
    }
    ops.add(OPS_LOG + OPS_EXP + OPS_LOG + OPS_EXP + 8.0 + 10.0 * (k + 1));
    return lead * sum;
}

// f(u) ~ (F(u + h) - F(u - h)) / (2h) with F the discretised distribution
// function of Eq. BEGE_LL_approx on the nodes w^j = w^0 + j dw, w^0 = 1e-4 -
// p s_p, dw = (10 s_p sqrt(p) - w^0) / (N - 1), and h = 1e-3 sqrt(s_p^2 p +
// s_n^2 n).  Both distribution functions share the increments
// dF_j = P(p, (w^j + p s_p)/s_p) - P(p, (w^{j-1} + p s_p)/s_p), so the
// difference is accumulated directly:
//   F(u + h) - F(u - h) = sum_j dF_j [P(n, y_j + d/2) - P(n, y_j - d/2)],
//   y_j = (w^{j-1} - u + n s_n) / s_n,  d = 2h / s_n,
// where the bracket is the Gamma(n, 1) mass of [y_j - d/2, y_j + d/2]:
// zero when the interval lies below 0, the Taylor form above when the
// interval is short against the density's scale (the usual case: d is 2e-3
// standard deviations of u over s_n), else the difference of the two
// incomplete gamma values: of Q = 1 - P when both ends lie in the upper tail
// (y >= n + 1, where the two P would be within rounding of 1), the termwise
// integral near 0 (y <= 2), else of P.  Nodes with dF_j = 0 (where P(p, .) has
// saturated) add nothing.
template <bool COUNT>
__device__ double bege_density(double u, double p, double n, double sp, double sn, int n_omega,
                               OpCount<COUNT> &ops)
{
    const double h = 1e-3 * sqrt(sp * sp * p + sn * sn * n);
    const double w0 = 1e-4 - p * sp;
    const double dw = (10.0 * sp * sqrt(p) - w0) / (n_omega - 1);
    const double lgp = lgamma(p), lgn = lgamma(n);
    const double psp = p * sp, nsn = n * sn;
    const double c = n - 1.0;
    const double zc = 1.0 + sqrt(fabs(c));
    const double d = 2.0 * h / sn;
    // node positions by multiplication with the scales' reciprocals: within
    // an ulp or two of the quotients, like the rounding of the nodes
    // themselves
    const double rsp = 1.0 / sp, rsn = 1.0 / sn;
    ops.add(2.0 * OPS_LGAMMA + 32.0);
    // The increments of P(p, .) over the nodes.  Where the Taylor series of
    // the density converges fast (gamma_taylor), the increment is the
    // density's integral over the interval, the density being carried from
    // node to node by the same series (evaluated directly where a run of such
    // intervals starts, and again before it would reach the denormals).
    // Elsewhere (the first nodes, whose intervals reach too close to 0, and
    // where the log-density changes fast): below x = p + 1 as the difference
    // of two P (series), above it as the difference of two Q (continued
    // fraction), where the two P would be within rounding of 1; the one
    // increment that crosses p + 1 as (1 - Q) - P.
    const double am1 = p - 1.0;
    const double xsplit = p + 1.0;
    double x = (w0 + psp) * rsp;
    bool have_prev = false, upper = false, have_g = false;
    double prev = 0.0, g = 0.0;
    double acc = 0.0;
    for (int j = 1; j <= n_omega; ++j) {
        const double xn = (w0 + j * dw + psp) * rsp;
        const double dx = xn - x;
        ops.add(6.0);
        double dF = 0.0;
        bool done = false;
        const bool left = x < am1;
        const double X = left ? x : xn;
        if (X > 0.0 && dx > 0.0) {
            const double rX = recip(X);
            const double beta = dx * rX;
            const double l1 = fabs(fma(am1, rX, -1.0)) * dx;
            ops.add(8.0);
            if (beta <= 0.5 && l1 <= TAYLOR_L1 && fabs(am1) * beta * beta <= TAYLOR_CURV) {
                if (!have_g) {
                    g = exp(am1 * log(x) - x - lgp);  // the density at x
                    have_g = true;
                    ops.add(OPS_LOG + OPS_EXP + 3.0);
                }
                const double sg = left ? -1.0 : 1.0;
                const TaylorSum ts = gamma_taylor(sg * (X - am1), beta, dx, sg, ops);
                if (ts.ok) {
                    if (left) {
                        dF = g * dx * ts.I;
                        g *= ts.H;
                    } else {
                        g *= recip(ts.H);
                        dF = g * dx * ts.I;
                    }
                    ops.add(3.0);
                    have_g = g > 0x1p-1000;
                    have_prev = false;
                    done = true;
                }
            }
        }
        if (!done) {
            have_g = false;
            if (!have_prev) {
                upper = x >= xsplit;
                prev = upper ? igam_q_upper(p, x, lgp, ops) : igam_p(p, x, lgp, ops);
                have_prev = true;
            }
            if (xn >= xsplit) {
                const double q = igam_q_upper(p, xn, lgp, ops);
                dF = upper ? prev - q : (1.0 - q) - prev;
                prev = q;
                upper = true;
            } else {
                const double pv = igam_p(p, xn, lgp, ops);
                dF = pv - prev;
                prev = pv;
            }
        }
        x = xn;
        if (dF == 0.0)
            continue;
        const double base = w0 + (j - 1) * dw - u + nsn;
        const double yhi = (base + h) * rsn;
        if (!(yhi > 0.0))
            continue;
        const double ylo = (base - h) * rsn;
        const double ym = base * rsn;
        const double v = recip(ym);
        const double L1 = c * v - 1.0;
        const double z = d * (fabs(L1) + zc * v);
        double mass;
        ops.add(17.0);
        if (ylo > 0.0 && z <= 0.03) {
            mass = gamma_mass_taylor(c, ym, v, L1, d, lgn);
            ops.add(OPS_TAYLOR);
        } else if (ylo >= n + 1.0) {
            // both ends in the upper tail: the difference of the two upper
            // functions, each with its full relative accuracy
            mass = igam_q_upper(n, ylo, lgn, ops) - igam_q_upper(n, yhi, lgn, ops);
        } else if (yhi <= 2.0) {
            // near 0: the termwise integral (for a small shape both P are
            // near 1 there)
            mass = gamma_mass_low(n, ylo, yhi, lgn, ops);
        } else {
            mass = igam_p(n, yhi, lgn, ops) - igam_p(n, ylo, lgn, ops);
        }
        acc += dF * mass;
    }
    return acc / (2.0 * h);
}

template <bool COUNT>
__global__ __launch_bounds__(DENSITY_BLOCK) void k_bege_density(BegeBatch b)
{
    const int chunk = b.chunk_order[blockIdx.x];
    const int k = chunk / b.chunks;
    const int t = (chunk - k * b.chunks) * DENSITY_BLOCK + threadIdx.x + 1;
    OpCount<COUNT> ops;
    if (t <= b.T) {
        const double *th = b.theta + static_cast<size_t>(k) * BEGE_NPAR;
        const double sp = th[SP], sn = th[SN], mu = th[MU];
        const size_t o = static_cast<size_t>(k) * b.T + (t - 1);
        const double p = b.shape_p[o], n = b.shape_n[o];
        double out = -INFINITY;
        if (sp > 0.0 && sn > 0.0 && p > 0.0 && n > 0.0) {
            const double f = bege_density(b.r[t] - mu, p, n, sp, sn, b.n_omega, ops);
            ops.add(OPS_LOG + 2.0);
            if (f > 0.0)
                out = log(f);
        }
        b.logdens[o] = out;
    }
    if constexpr (COUNT) {
        // integer-valued totals: exact in any order
        double v = ops.v;
        for (int m = 32; m > 0; m >>= 1)
            v += __shfl_xor(v, m, 64);
        if (threadIdx.x == 0)
            atomicAdd(b.ops, v);
    }
}

__global__ __launch_bounds__(SUM_BLOCK) void k_bege_sum(BegeBatch b)
{
    __shared__ double s[SUM_BLOCK];
    const int k = blockIdx.x;
    const double *ld = b.logdens + static_cast<size_t>(k) * b.T;
    double v = 0.0;
    for (int t = threadIdx.x; t < b.T; t += SUM_BLOCK)
        v += ld[t];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = SUM_BLOCK / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        b.loglik[k] = s[0];
}

}  // namespace

int bege_chunks(int T)
{
    return (T + DENSITY_BLOCK - 1) / DENSITY_BLOCK;
}

hipError_t launch_bege(const BegeBatch &b, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    hipLaunchKernelGGL(k_bege_shapes, dim3(b.n_theta), dim3(SHAPES_BLOCK), 0, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_bege_order, dim3(1), dim3(ORDER_BLOCK), 0, s, b);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    const uint64_t grid = static_cast<uint64_t>(b.chunks) * b.n_theta;
    if (ev0)
        (void)hipEventRecord(ev0, s);
    if (b.ops)
        hipLaunchKernelGGL(k_bege_density<true>, dim3(static_cast<unsigned>(grid)), dim3(DENSITY_BLOCK),
                           0, s, b);
    else
        hipLaunchKernelGGL(k_bege_density<false>, dim3(static_cast<unsigned>(grid)),
                           dim3(DENSITY_BLOCK), 0, s, b);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (ev1)
        (void)hipEventRecord(ev1, s);
    hipLaunchKernelGGL(k_bege_sum, dim3(b.n_theta), dim3(SUM_BLOCK), 0, s, b);
    return hipGetLastError();
}

}  // namespace pps
