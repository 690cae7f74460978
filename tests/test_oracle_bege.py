"""Pins of the oracle's BEGE log-likelihood (Sec. 4.2: Eqs. BEGE, shape,
BEGE_LL, CDF_BEGE, BEGE_LL_approx, incompGamma) against facts fixed outside
its code:

* P(a, x) equals scipy's regularised incomplete gamma function, across both
  of its branches and for shapes up to 1e7 (where the leading factor loses
  about a ln(a) ulps);
* the discretised distribution function: as sigma_n -> 0 the negative shock
  vanishes and the sum telescopes to F_X(first node >= u) - F_X(w^0); for
  sigma_n > 0 it is the left-node Riemann-Stieltjes sum of the exact integral
  of Eq. CDF_BEGE over the grid, so it lies between that integral (computed
  by adaptive quadrature over scipy's gamma laws) and the right-node sum, and
  the gap shrinks like the grid spacing;
* the density: on fine grids it converges to the exact convolution density of
  u = s_p w_p - s_n w_n restricted to the grid's range;
* the log-likelihood: with rho = phi = 0 the shapes stay at (p0, n0); with
  phi = 0 they follow p0 (1 - rho^t) / (1 - rho); the asymmetric terms follow
  the sign of u (Eq. shape); a non-positive shape gives -inf;
* the simulator's shocks are centred gamma variates (KS test against scipy).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
import pps_workloads as W

EPS = 2.0 ** -52


def gamma_tol(a, x):
    """Absolute error allowance of P(a, x): the leading factor
    exp(-x + a ln x - ln Gamma(a)) is formed from terms of size up to
    x + a |ln x| + |ln Gamma(a)|, each rounded to about one ulp."""
    big = x + a * abs(math.log(max(x, 1e-300))) + abs(math.lgamma(a))
    return 64.0 * EPS * (1.0 + big)


@pytest.mark.parametrize("a", [1e-4, 0.05, 0.3, 1.0, 2.5, 10.0, 100.0, 1e4, 1e6, 1e7])
def test_gamma_p_matches_scipy(a):
    xs = [0.0, 1e-8, 1e-3, 0.5, 1.0, 5.0, 40.0]
    xs += [a * f for f in (1e-3, 0.1, 0.5, 0.9, 0.99, 1.0, 1.01, 1.1, 2.0, 10.0)]
    xs += [a + 1.0 - 1e-9, a + 1.0, a + 1.0 + 1e-9, a + 3.0 * math.sqrt(a), a - 3.0 * math.sqrt(a)]
    for x in xs:
        if x < 0.0:
            continue
        ref = special.gammainc(a, x)
        got = oracle.gamma_p(a, x)
        assert abs(got - ref) <= gamma_tol(a, x) + 1e-15 * ref, (a, x, got, ref)
        # small values to relative accuracy
        if 0.0 < ref < 1e-3:
            assert abs(got / ref - 1.0) < 1e-12 + gamma_tol(a, x) * 1e3, (a, x, got, ref)


def grid(p, sp, n_omega):
    """The paper's quadrature nodes w^0..w^N (Sec. 4.2, experiment settings)."""
    w0 = 1e-4 - p * sp
    dw = (10.0 * sp * math.sqrt(p) - w0) / (n_omega - 1)
    return w0 + dw * np.arange(n_omega + 1)


def laws(p, n, sp, sn):
    """X = s_p (G_p - p) and Y = s_n (G_n - n): centred gamma laws."""
    return stats.gamma(p, loc=-p * sp, scale=sp), stats.gamma(n, loc=-n * sn, scale=sn)


@pytest.mark.parametrize("p,sp", [(0.3, 0.02), (3.0, 0.01), (40.0, 0.05)])
def test_cdf_without_negative_shocks_telescopes(p, sp):
    X, _ = laws(p, 1.0, sp, 1e-9)
    nodes = grid(p, sp, 100)
    for j in (3, 17, 50, 98):
        u = 0.5 * (nodes[j] + nodes[j + 1])     # strictly between two nodes
        got = oracle.bege_cdf(u, p, 2.0, sp, 1e-9, 100)
        ref = X.cdf(nodes[j + 1]) - X.cdf(nodes[0])
        assert abs(got - ref) < 1e-12, (j, got, ref)
    # below the grid nothing is counted; above it, all of it
    assert oracle.bege_cdf(nodes[0] - sp, p, 2.0, sp, 1e-9, 100) == 0.0
    top = oracle.bege_cdf(nodes[-1] + sp, p, 2.0, sp, 1e-9, 100)
    assert abs(top - (X.cdf(nodes[-1]) - X.cdf(nodes[0]))) < 1e-12


CASES = [(0.3, 0.6, 0.02, 0.03, 0.01), (3.0, 2.0, 0.01, 0.02, -0.02),
         (12.0, 0.8, 0.015, 0.05, 0.03), (1.5, 25.0, 0.04, 0.01, 0.0)]


def exact_grid_cdf(u, p, n, sp, sn, lo, hi):
    """Eq. CDF_BEGE with the outer integral restricted to [lo, hi]."""
    X, Y = laws(p, n, sp, sn)
    f = lambda x: Y.sf(x - u) * X.pdf(x)
    # break the range at the mode of X and at the tail's transition
    pts = sorted(v for v in (max(p - 1.0, 0.0) * sp - p * sp, u) if lo < v < hi)
    return integrate.quad(f, lo, hi, points=pts or None, limit=400, epsabs=1e-14, epsrel=1e-12)[0]


@pytest.mark.parametrize("p,n,sp,sn,u", CASES)
def test_cdf_is_the_left_node_sum_of_the_integral(p, n, sp, sn, u):
    X, Y = laws(p, n, sp, sn)
    gaps = []
    for n_omega in (100, 400, 1600):
        nodes = grid(p, sp, n_omega)
        got = oracle.bege_cdf(u, p, n, sp, sn, n_omega)
        exact = exact_grid_cdf(u, p, n, sp, sn, nodes[0], nodes[-1])
        # the tail 1 - F_Y(w - u) falls as w rises, so the sum with the tail
        # taken at each cell's left node is an upper sum, the right-node one a
        # lower sum, of the exact integral
        lower = np.sum(Y.sf(nodes[1:] - u) * np.diff(X.cdf(nodes)))
        assert lower - 1e-12 <= exact <= got + 1e-12, (n_omega, lower, exact, got)
        gaps.append(got - exact)
    assert gaps[2] < 0.5 * gaps[0] + 1e-12


@pytest.mark.parametrize("p,n,sp,sn,u", [c for c in CASES if min(c[0], c[1]) >= 1.0])
def test_density_converges_to_the_convolution(p, n, sp, sn, u):
    """The density estimate differentiates the left-node sum, whose error is
    first order in the spacing; Richardson's combination 2 D(2N) - D(N) of
    two grids removes that term and must land on the exact density of u
    (the convolution of the two centred gamma laws over the grid's range) to
    second order.  A one-sided difference in place of the central one would
    leave a bias of order h f'/f, about 1e-3 of the density."""
    X, Y = laws(p, n, sp, sn)
    nodes = grid(p, sp, 4000)
    f = lambda x: X.pdf(x) * Y.pdf(x - u)
    exact = integrate.quad(f, nodes[0], nodes[-1], points=[u], limit=800, epsabs=1e-14,
                           epsrel=1e-12)[0]
    d1 = oracle.bege_density(u, p, n, sp, sn, 2000)
    d2 = oracle.bege_density(u, p, n, sp, sn, 4000)
    assert abs(d2 / exact - 1.0) < 2e-3, (d2, exact)
    assert abs((2.0 * d2 - d1) / exact - 1.0) < 2e-5, (d1, d2, exact)
    # at the paper's N_omega = 100 the estimate is still the right size
    assert abs(oracle.bege_density(u, p, n, sp, sn, 100) / exact - 1.0) < 0.1


@pytest.fixture(scope="module")
def series():
    return np.array(W.BEGE_THETA_OBS), oracle.bege_simulate(W.BEGE_THETA_OBS, 200, 11)


def test_loglik_constant_shapes(series):
    th, r = series
    th = th.copy()
    th[[2, 3, 4, 7, 8, 9]] = 0.0          # rho = phi = 0: p_t = p0, n_t = n0
    o = oracle.bege_loglik(th, r)
    for t in (1, 2, 50, 200):
        f = oracle.bege_density(r[t] - th[10], th[0], th[5], th[1], th[6], 100)
        assert o["logdens"][t - 1] == math.log(f)
    assert o["loglik"] == pytest.approx(o["logdens"].sum(), rel=1e-14)


def test_loglik_geometric_shapes(series):
    th, r = series
    th = th.copy()
    th[[3, 4, 8, 9]] = 0.0                # phi = 0: u_t meets p_{t-1} = p0 (1 - rho^t) / (1 - rho)
    o = oracle.bege_loglik(th, r)
    for t in (1, 2, 7, 60, 200):
        p = th[0] * (1.0 - th[2] ** t) / (1.0 - th[2])
        n = th[5] * (1.0 - th[7] ** t) / (1.0 - th[7])
        f = oracle.bege_density(r[t] - th[10], p, n, th[1], th[6], 100)
        assert o["logdens"][t - 1] == pytest.approx(math.log(f), rel=1e-9, abs=1e-9)


def test_loglik_asymmetric_shapes():
    # theta = (p0, s_p, rho_p, phi_p+, phi_p-, n0, s_n, rho_n, phi_n+, phi_n-, mu)
    th = np.array([0.4, 0.03, 0.5, 0.2, 0.05, 0.3, 0.02, 0.6, -0.01, 0.3, 0.01])
    r = np.array([0.0, 0.01 + 0.06, 0.01 - 0.05, 0.01 + 0.02])   # u_1 > 0, u_2 < 0
    o = oracle.bege_loglik(th, r)
    u1, u2 = 0.06, -0.05
    p1 = th[0] + th[2] * th[0] + th[3] * u1 * u1 / (2 * th[1] ** 2)
    n1 = th[5] + th[7] * th[5] + th[8] * u1 * u1 / (2 * th[6] ** 2)
    p2 = th[0] + th[2] * p1 + th[4] * u2 * u2 / (2 * th[1] ** 2)
    n2 = th[5] + th[7] * n1 + th[9] * u2 * u2 / (2 * th[6] ** 2)
    for t, (p, n) in enumerate([(th[0], th[5]), (p1, n1), (p2, n2)], start=1):
        f = oracle.bege_density(r[t] - th[10], p, n, th[1], th[6], 100)
        assert o["logdens"][t - 1] == pytest.approx(math.log(f), rel=1e-12)
    # a negative phi_n+ that drives n_t below zero: that step and the
    # log-likelihood are -inf, earlier steps are unaffected
    th2 = th.copy()
    th2[8] = -0.2
    r2 = np.array([0.0, 0.01 + 0.1, 0.01, 0.01])
    n1 = th2[5] + th2[7] * th2[5] + th2[8] * 0.01 / (2 * th2[6] ** 2)
    assert n1 < 0
    o2 = oracle.bege_loglik(th2, r2)
    assert np.isfinite(o2["logdens"][0]) and o2["logdens"][1] == -np.inf
    assert o2["loglik"] == -np.inf


def test_loglik_batch_equals_single_calls(series):
    _, r = series
    th = W.bege_prior_draws(12, seed=3)
    batch = oracle.bege_loglik_batch(th, r)
    one = np.array([oracle.bege_loglik(t, r)["loglik"] for t in th])
    np.testing.assert_array_equal(batch, one)


@pytest.mark.parametrize("shape", [0.3, 2.5])
def test_simulated_shocks_are_centred_gamma(shape):
    # rho = phi = 0 and a vanishing negative scale: r_t - mu = s_p (G - p0)
    th = np.array([shape, 0.02, 0.0, 0.0, 0.0, 1.0, 1e-12, 0.0, 0.0, 0.0, 0.01])
    r = oracle.bege_simulate(th, 4000, 5)
    X = stats.gamma(shape, loc=-shape * 0.02, scale=0.02)
    assert stats.kstest(r - 0.01, X.cdf).pvalue > 1e-3
    # and the negative shocks mirror them
    th2 = np.array([1.0, 1e-12, 0.0, 0.0, 0.0, shape, 0.03, 0.0, 0.0, 0.0, 0.0])
    r2 = oracle.bege_simulate(th2, 4000, 6)
    Y = stats.gamma(shape, loc=-shape * 0.03, scale=0.03)
    assert stats.kstest(-r2, Y.cdf).pvalue > 1e-3


def test_observed_series_is_the_golden_one():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "observed.json")) as f:
        g = json.load(f)["bege_T1099"]
    r = oracle.bege_simulate(g["theta"], g["T"], g["seed"])
    np.testing.assert_array_equal(r, np.array(g["r"]))
    assert abs(r.std() - 0.057) < 0.01


# ---- the upper tail and the quad-precision difference ----------------------

def _mp_gamma(a, x, upper):
    import mpmath as mp
    return mp.gammainc(mp.mpf(a), mp.mpf(x), mp.inf, regularized=True) if upper else \
        mp.gammainc(mp.mpf(a), 0, mp.mpf(x), regularized=True)


@pytest.mark.parametrize("a,x", [(0.008, 64.0), (0.83, 676.0), (49.7, 135.0), (0.3, 2.0),
                                 (5.0, 6.0), (2.0, 700.0), (1e3, 1.3e3)])
def test_gamma_q_upper_tail_relative(a, x):
    """Q(a, x) = 1 - P(a, x) keeps its relative accuracy down to e^-700
    (50-digit mpmath); P = 1 - Q stays consistent."""
    import mpmath as mp
    mp.mp.dps = 50
    ref = float(_mp_gamma(a, x, True))
    got = oracle.gamma_q(a, x)
    assert abs(got / ref - 1.0) < 1e-12 + gamma_tol(a, x) * 10, (a, x, got, ref)
    assert oracle.gamma_p(a, x) == 1.0 - got


def _mp_density(u, p, n, sp, sn, n_omega, dps=50):
    """The central difference of the discretised distribution function of
    Eq. BEGE_LL_approx (as the oracle reads it: nodes w^j, h = 1e-3 sd), the
    two sums formed as written and subtracted, at `dps` digits."""
    import mpmath as mp
    mp.mp.dps = dps
    p, n, sp, sn, u = (mp.mpf(v) for v in (p, n, sp, sn, u))
    w0 = mp.mpf('1e-4') - p * sp
    dw = (10 * sp * mp.sqrt(p) - w0) / (n_omega - 1)

    def cdf(uu):
        prev = _mp_gamma(p, (w0 + p * sp) / sp, False)
        f = mp.mpf(0)
        for j in range(1, n_omega + 1):
            cur = _mp_gamma(p, (w0 + j * dw + p * sp) / sp, False)
            x = (w0 + (j - 1) * dw - uu + n * sn) / sn
            tail = _mp_gamma(n, x, True) if x > 0 else mp.mpf(1)
            f += tail * (cur - prev)
            prev = cur
        return f
    h = mp.mpf('1e-3') * mp.sqrt(sp * sp * p + sn * sn * n)
    return (cdf(u + h) - cdf(u - h)) / (2 * h)


# far left tails of u (the negative shock's upper tail): densities e^-27 .. e^-624,
# where the two FP64 sums agree to every bit; and an ordinary point
TAIL_CASES = [(-0.766984, 0.281325, 0.862055, 0.1061, 0.02371),
              (-0.715164, 0.490402, 0.00800925, 0.00508, 0.01121),
              (-0.486412, 0.243791, 49.7437, 0.2939, 0.005708),
              (0.01, 2.0, 3.0, 0.02, 0.03)]


@pytest.mark.parametrize("u,p,n,sp,sn", TAIL_CASES)
def test_density_in_the_tails_matches_50_digits(u, p, n, sp, sn):
    """The oracle's density (FP64, with the quad-precision difference where
    the FP64 one would keep fewer than ~20 bits) and the quad evaluation
    itself against the same formula at 50 digits (N_omega = 12)."""
    ref = float(_mp_density(u, p, n, sp, sn, 12))
    assert ref > 0.0
    q = oracle.bege_density_q(u, p, n, sp, sn, 12)
    f = oracle.bege_density(u, p, n, sp, sn, 12)
    assert abs(q / ref - 1.0) < 1e-14, (q, ref)
    assert abs(f / ref - 1.0) < 1e-6, (f, ref)


def test_density_n_omega_100_deep_tail():
    """One deep-tail point at the benchmark's N_omega = 100: log f = -68.41
    (the literal FP64 difference is exactly 0 there)."""
    u, p, n, sp, sn = TAIL_CASES[1]
    ref = float(_mp_density(u, p, n, sp, sn, 100))
    f = oracle.bege_density(u, p, n, sp, sn, 100)
    assert abs(math.log(f) - math.log(ref)) < 1e-10, (math.log(f), math.log(ref))


def test_density_where_the_two_sums_agree_beyond_quad_precision():
    """A huge positive-shock shape (grid spacing ~1 sd of its law): F(u + h)
    and F(u - h) are ~0.9 and differ by ~1e-39 (log f = -83.65), beyond the
    113 bits of a quad difference of the two sums; the oracle's quad tier
    regroups the difference by node.  Against the literal formula at 90
    digits, N_omega = 100."""
    u, p, n, sp, sn = 0.0151, 8376.36, 0.426262, 0.0226767, 0.0192717
    ref = _mp_density(u, p, n, sp, sn, 100, dps=90)
    f = oracle.bege_density(u, p, n, sp, sn, 100)
    assert abs(math.log(f) - float(mp_log(ref))) < 1e-10, (math.log(f), float(mp_log(ref)))


def mp_log(v):
    import mpmath as mp
    return mp.log(v)
