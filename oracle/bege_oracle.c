/*
 * FP64 CPU oracle for the log-likelihood of the BEGE volatility model of
 * Sec. 4.2 (Warne, Sisson & Drovandi, arXiv:1902.09046): returns driven by
 * positive and negative centred-gamma shocks (Eq. BEGE) whose shapes follow
 * the recursions of Eq. shape; transition densities by finite differences of
 * the BEGE distribution function (Eq. CDF_BEGE) discretised as in
 * Eq. BEGE_LL_approx, with the regularised incomplete gamma function of
 * Eq. incompGamma; log-likelihood Eq. BEGE_LL.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against; nothing in the product path may link, load
 * or call it, and it shares no code with the HIP library.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>

/* from pps_oracle.c */
void or_stream_block(uint64_t seed, uint64_t draw, uint32_t block, uint32_t purpose,
                     uint32_t out[4]);
double or_uniform(uint32_t word);
void or_box_muller(uint32_t w0, uint32_t w1, double *z0, double *z1);

#define OR_BEGE_NPAR 11
#define OR_IGAM_MAXIT 100000
#define OR_IGAM_EPS 1.1102230246251565e-16 /* 2^-53 */

/* Regularised lower incomplete gamma P(a, x) (Eq. incompGamma), x >= 0:
 *   x < a + 1: the power series P = e^-x x^a sum_{k>=0} x^k / Gamma(a + k + 1),
 *     summed as (1/a) (1 + x/(a+1) + x^2/((a+1)(a+2)) + ...) until a term is
 *     below 2^-53 of the sum;
 *   x >= a + 1: P = 1 - Q with the continued fraction of the upper function
 *     Gamma(a, x) = e^-x x^a / (x + 1 - a - 1 (1 - a) / (x + 3 - a - 2 (2 - a)
 *     / (x + 5 - a - ...))), evaluated by the modified Lentz method until a
 *     factor is within 2^-53 of 1 (the series alone would overflow for large
 *     x: its terms grow like e^x before they fall).
 * x <= 0 gives 0.                                                           */
/* P(a, x) and its complement Q(a, x) = 1 - P(a, x) (*q): the series gives P
 * and Q = 1 - P; the continued fraction gives Q = lead * fraction directly
 * and P = 1 - Q, so a Q of e^-x size keeps its relative accuracy.          */
static double gamma_pq(double a, double x, double *q)
{
    if (!(x > 0.0)) {
        *q = 1.0;
        return 0.0;
    }
    const double lead = exp(-x + a * log(x) - lgamma(a));
    if (x < a + 1.0) {
        double term = 1.0 / a, sum = term, den = a;
        for (int k = 1; k < OR_IGAM_MAXIT; ++k) {
            den += 1.0;
            term *= x / den;
            sum += term;
            if (fabs(term) < fabs(sum) * OR_IGAM_EPS)
                break;
        }
        const double pv = sum * lead;
        *q = 1.0 - pv;
        return pv;
    }
    const double tiny = 1e-300;
    double b = x + 1.0 - a;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double f = d;
    for (int i = 1; i < OR_IGAM_MAXIT; ++i) {
        const double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (fabs(d) < tiny)
            d = tiny;
        c = b + an / c;
        if (fabs(c) < tiny)
            c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        f *= del;
        if (fabs(del - 1.0) < OR_IGAM_EPS)
            break;
    }
    *q = lead * f;
    return 1.0 - *q;
}

double or_gamma_p(double a, double x)
{
    double q;
    return gamma_pq(a, x, &q);
}

/* Q(a, x) = 1 - P(a, x), the upper regularised incomplete gamma function. */
double or_gamma_q(double a, double x)
{
    double q;
    gamma_pq(a, x, &q);
    return q;
}

/* Distribution function of u = s_p w_p - s_n w_n, w ~ centred gamma (shapes p,
 * n), by the discretised integral of Eq. BEGE_LL_approx on the grid of the
 * paper: w^j = w^0 + j dw, j = 0..N, w^0 = 1e-4 - p s_p, dw = (10 s_p sqrt(p)
 * - w^0) / (N - 1):
 *   F(u) = sum_{j=1..N} [1 - P(n, (w^{j-1} - u + n s_n)/s_n)]
 *                       [P(p, (w^j + p s_p)/s_p) - P(p, (w^{j-1} + p s_p)/s_p)].
 * The first factor is the upper function Q(n, .), taken as computed (not as
 * 1 minus a P that is within rounding of 1).                                */
double or_bege_cdf(double u, double p, double n, double sp, double sn, int n_omega)
{
    const double w0 = 1e-4 - p * sp;
    const double dw = (10.0 * sp * sqrt(p) - w0) / (n_omega - 1);
    double prev = or_gamma_p(p, (w0 + p * sp) / sp);
    double f = 0.0;
    for (int j = 1; j <= n_omega; ++j) {
        const double wj = w0 + j * dw, wjm = w0 + (j - 1) * dw;
        const double cur = or_gamma_p(p, (wj + p * sp) / sp);
        const double tail = or_gamma_q(n, (wjm - u + n * sn) / sn);
        f += tail * (cur - prev);
        prev = cur;
    }
    return f;
}

/* ---- the same difference in quad precision (__float128: 113-bit
 * significand), for the steps where the two FP64 sums of the central
 * difference cancel.                                                        */
typedef __float128 quad;
#define OR_IGAM_EPS_Q 1.925929944387235853055977942584927319e-34Q /* 2^-112 */

/* P and Q as gamma_pq, in quad precision. */
static quad gamma_pq_q(quad a, quad x, quad *q)
{
    if (!(x > 0)) {
        *q = 1;
        return 0;
    }
    const quad lead = expq(-x + a * logq(x) - lgammaq(a));
    if (x < a + 1) {
        quad term = 1 / a, sum = term, den = a;
        for (int k = 1; k < OR_IGAM_MAXIT; ++k) {
            den += 1;
            term *= x / den;
            sum += term;
            if (fabsq(term) < fabsq(sum) * OR_IGAM_EPS_Q)
                break;
        }
        *q = 1 - sum * lead;
        return sum * lead;
    }
    const quad tiny = 1e-4000Q;
    quad b = x + 1 - a;
    quad c = 1 / tiny;
    quad d = 1 / b;
    quad f = d;
    for (int i = 1; i < OR_IGAM_MAXIT; ++i) {
        const quad an = -i * (i - a);
        b += 2;
        d = an * d + b;
        if (fabsq(d) < tiny)
            d = tiny;
        c = b + an / c;
        if (fabsq(c) < tiny)
            c = tiny;
        d = 1 / d;
        const quad del = d * c;
        f *= del;
        if (fabsq(del - 1) < OR_IGAM_EPS_Q)
            break;
    }
    *q = lead * f;
    return 1 - *q;
}

/* F(u + h) - F(u - h) in quad precision, summed node by node:
 *   sum_j [P(p, x_j) - P(p, x_{j-1})] [Q(n, y_j(u + h)) - Q(n, y_j(u - h))],
 * the difference of the two sums of Eq. BEGE_LL_approx regrouped by node
 * (the increments of P(p, .) are common to both).  Each difference of two
 * values of the complementary pair (P, Q) is taken on the side where the two
 * values are small: of P below the argument a + 1, of Q above it, so terms
 * whose two values agree to more than quad precision (F(u + h) and F(u - h)
 * near 1/2 with a difference of e^-100) keep their significant digits.     */
static quad pair_diff_q(quad a, quad xlo, quad xhi)
{
    /* P(a, xhi) - P(a, xlo) = Q(a, xlo) - Q(a, xhi), xlo <= xhi, P = 0 below 0 */
    quad qlo, qhi;
    const quad plo = gamma_pq_q(a, xlo, &qlo);
    const quad phi = gamma_pq_q(a, xhi, &qhi);
    return xlo >= a + 1 ? qlo - qhi : phi - plo;
}

static quad bege_cdf_diff_q(quad u, quad h, quad p, quad n, quad sp, quad sn, int n_omega)
{
    const quad w0 = 1e-4Q - p * sp;
    const quad dw = (10 * sp * sqrtq(p) - w0) / (n_omega - 1);
    quad d = 0;
    for (int j = 1; j <= n_omega; ++j) {
        const quad wj = w0 + j * dw, wjm = w0 + (j - 1) * dw;
        const quad dF = pair_diff_q(p, (wjm + p * sp) / sp, (wj + p * sp) / sp);
        /* y_j(u + h) <= y_j(u - h): the tails differ by the Gamma(n) mass between */
        const quad m = pair_diff_q(n, (wjm - (u + h) + n * sn) / sn, (wjm - (u - h) + n * sn) / sn);
        d += dF * m;
    }
    return d;
}

/* The central difference below in quad precision (regrouped by node). */
double or_bege_density_q(double u, double p, double n, double sp, double sn, int n_omega)
{
    const quad h = 1e-3Q * sqrtq((quad)sp * sp * p + (quad)sn * sn * n);
    return (double)(bege_cdf_diff_q(u, h, p, n, sp, sn, n_omega) / (2 * h));
}

/* Transition density by the central difference (F(u + h) - F(u - h)) / (2 h),
 * h = 1e-3 times the standard deviation sqrt(s_p^2 p + s_n^2 n) of u.  Each
 * distribution function is a sum of N_omega products of factors in [0, 1]
 * (a tail 1 - P and an increment of P), so in FP64 it carries an absolute
 * rounding error of about N_omega ulps of 1 whatever its own size.  Where the
 * difference is below 2^-26 that error would leave it fewer than ~20 correct
 * bits, so it is evaluated again in quad precision, regrouped by node.      */
double or_bege_density(double u, double p, double n, double sp, double sn, int n_omega)
{
    const double h = 1e-3 * sqrt(sp * sp * p + sn * sn * n);
    const double fp = or_bege_cdf(u + h, p, n, sp, sn, n_omega);
    const double fm = or_bege_cdf(u - h, p, n, sp, sn, n_omega);
    if (fabs(fp - fm) <= 0x1p-26)
        return or_bege_density_q(u, p, n, sp, sn, n_omega);
    return (fp - fm) / (2.0 * h);
}

/* log L(theta; r_0..r_T) of Eq. BEGE_LL, theta = (p0, s_p, rho_p, phi_p+,
 * phi_p-, n0, s_n, rho_n, phi_n+, phi_n-, mu):
 *   shapes at t = 0 are the initial conditions p0, n0;
 *   for t = 1..T: u_t = r_t - mu; log f(u_t | p_{t-1}, n_{t-1}); then
 *     p_t = p0 + rho_p p_{t-1} + phi_p^{+/-} u_t^2 / (2 s_p^2)  (+ for u_t >= 0),
 *     n_t = n0 + rho_n n_{t-1} + phi_n^{+/-} u_t^2 / (2 s_n^2)   (Eq. shape).
 * A non-positive shape or density estimate gives log f = -inf at that step.
 * The shocks of Eq. BEGE are s_p w_p - s_n w_n with w_p, w_n gamma variates
 * of unit scale, so s_p and s_n are the scales of gamma laws: a law with a
 * scale that is not positive does not exist, such a theta lies outside the
 * model's parameter space, and its likelihood is zero (log f = -inf at every
 * step).  ld (optional, T values) receives each log f.  Returns 0.          */
int or_bege_loglik(const double *th, const double *r, int T, int n_omega, double *ld, double *ll)
{
    const double p0 = th[0], sp = th[1], rp = th[2], ppos = th[3], pneg = th[4];
    const double n0 = th[5], sn = th[6], rn = th[7], npos = th[8], nneg = th[9], mu = th[10];
    const int scales_ok = sp > 0.0 && sn > 0.0;
    double p = p0, n = n0, acc = 0.0;
    for (int t = 1; t <= T; ++t) {
        const double u = r[t] - mu;
        double lf = -INFINITY;
        if (scales_ok && p > 0.0 && n > 0.0) {
            const double f = or_bege_density(u, p, n, sp, sn, n_omega);
            lf = f > 0.0 ? log(f) : -INFINITY;
        }
        if (ld)
            ld[t - 1] = lf;
        acc += lf;
        const double u2 = u * u;
        p = p0 + rp * p + (u >= 0.0 ? ppos : pneg) * u2 / (2.0 * sp * sp);
        n = n0 + rn * n + (u >= 0.0 ? npos : nneg) * u2 / (2.0 * sn * sn);
    }
    *ll = acc;
    return 0;
}

/* Batched: log L of n_theta parameter vectors (rows of 11), OpenMP over rows;
 * ld (optional, n_theta x T, row k at k T) receives every step's log f.      */
int or_bege_loglik_batch(const double *theta, int n_theta, const double *r, int T, int n_omega,
                         double *ll, double *ld)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n_theta; ++k)
        or_bege_loglik(&theta[(size_t)k * OR_BEGE_NPAR], r, T, n_omega,
                       ld ? &ld[(size_t)k * T] : NULL, &ll[k]);
    return 0;
}

/* Gamma(a, 1) variate by the squeeze-and-reject method of Marsaglia and Tsang
 * (shape a >= 1; for a < 1 a draw of shape a + 1 times U^(1/a)).  Attempt k
 * of variate `id` uses block 2k (normal from words 0, 1; uniform word 2) and
 * the boost uniform comes from block 1 word 3.                               */
static double gamma_variate(double a, uint64_t seed, uint64_t id, uint32_t purpose)
{
    uint32_t w[4];
    double boost = 1.0;
    if (a < 1.0) {
        or_stream_block(seed, id, 1, purpose, w);
        boost = pow(or_uniform(w[3]), 1.0 / a);
        a += 1.0;
    }
    const double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
    for (uint32_t k = 0;; ++k) {
        or_stream_block(seed, id, 2 * k, purpose, w);
        double z, z1;
        or_box_muller(w[0], w[1], &z, &z1);
        const double v = 1.0 + c * z;
        if (v <= 0.0)
            continue;
        const double v3 = v * v * v;
        if (log(or_uniform(w[2])) < 0.5 * z * z + d - d * v3 + d * log(v3))
            return d * v3 * boost;
    }
}

/* A BEGE return series r_0..r_T at theta (Eq. BEGE with the shapes of Eq.
 * shape), consistent with the likelihood above: the shapes at t = 0 are
 * (p0, n0); for t = 1..T, u_t is drawn with shapes (p_{t-1}, n_{t-1}) and the
 * shapes are then updated with u_t.  r_0 (which the likelihood conditions on
 * and does not use) is drawn with the initial shapes.  w_p and w_n are centred
 * gamma variates (streams 0x80000000 and 0x80000001, variate index t).
 * Returns -1 if a shape becomes non-positive.                               */
int or_bege_simulate(const double *th, int T, uint64_t seed, double *r)
{
    const double p0 = th[0], sp = th[1], rp = th[2], ppos = th[3], pneg = th[4];
    const double n0 = th[5], sn = th[6], rn = th[7], npos = th[8], nneg = th[9], mu = th[10];
    double p = p0, n = n0;
    for (int t = 0; t <= T; ++t) {
        if (!(p > 0.0 && n > 0.0))
            return -1;
        const double wp = gamma_variate(p, seed, (uint64_t)t, 0x80000000u) - p;
        const double wn = gamma_variate(n, seed, (uint64_t)t, 0x80000001u) - n;
        const double u = sp * wp - sn * wn;
        r[t] = mu + u;
        if (t == 0)
            continue;
        const double u2 = u * u;
        p = p0 + rp * p + (u >= 0.0 ? ppos : pneg) * u2 / (2.0 * sp * sp);
        n = n0 + rn * n + (u >= 0.0 ? npos : nneg) * u2 / (2.0 * sn * sn);
    }
    return 0;
}
