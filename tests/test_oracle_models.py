"""Pins of the oracle's priors, simulators, ABC and p-values (CPU only).

Each check compares the oracle with something other than itself: a closed
form, an invariant, a library routine, or brute force on tiny inputs.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle
import pps_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "observed.json")


def _band(values, target, k=4.0):
    """|mean - target| within k standard errors."""
    se = values.std(ddof=1) / math.sqrt(len(values))
    return abs(values.mean() - target) <= k * se + 1e-15


# ---------------------------------------------------------------- priors ---

def test_uniform_priors_moments_and_bounds():
    spec = W.logistic_spec(steps=20, n_obs=20)
    th = np.array([oracle.prior_draw(spec, 3, i)[0] for i in range(20000)])
    for j, (lo, hi) in enumerate([(0, 2), (50, 150), (0, 0.5)]):
        assert th[:, j].min() > lo and th[:, j].max() < hi
        assert _band(th[:, j], (lo + hi) / 2)
        assert abs(th[:, j].var() - (hi - lo) ** 2 / 12) < 0.05 * (hi - lo) ** 2 / 12
    # parameters use distinct blocks: no correlation between them
    assert abs(np.corrcoef(th[:, 0], th[:, 1])[0, 1]) < 4 / math.sqrt(len(th))


def test_lognormal_and_normal_priors():
    lam = 0.7
    spec = W.logistic_spec(theta1=("lognormal", 0.3, lam))
    th1 = np.array([oracle.prior_draw(spec, 4, i)[0][0] for i in range(20000)])
    lg = np.log(th1)
    assert _band(lg, 0.3)
    assert abs(lg.std() - lam) < 0.03 * lam
    spec = W.normal_mean_spec(prior_sd=2.5)
    mu = np.array([oracle.prior_draw(spec, 4, i)[0][0] for i in range(20000)])
    assert _band(mu, 0.0)
    assert abs(mu.std() - 2.5) < 0.03 * 2.5


def test_point_prior_and_infinite_point():
    spec = W.logistic_spec(theta2=("point", math.inf, 0.0))
    th, att = oracle.prior_draw(spec, 1, 9)
    assert th[1] == math.inf and att == 1


def test_garch_constraint_acceptance_closed_form():
    """P(alpha + beta < 1) for alpha ~ U(0, .3), beta ~ U(.5, .99) is
    (0.01 + (0.5*0.29 - (0.3^2 - 0.01^2)/2)/0.49)/0.3 = 0.713946."""
    p = (0.01 + (0.5 * 0.29 - (0.3**2 - 0.01**2) / 2) / 0.49) / 0.3
    assert abs(p - 0.71395) < 1e-5
    spec = W.garch_spec()
    n = 40000
    att = np.array([oracle.prior_draw(spec, 7, i)[1] for i in range(n)])
    first = (att == 1).mean()
    assert abs(first - p) <= 4 * math.sqrt(p * (1 - p) / n)
    # attempts are geometric with success probability p
    assert abs(att.mean() - 1 / p) < 4 * math.sqrt((1 - p) / p**2 / n)
    th = np.array([oracle.prior_draw(spec, 7, i)[0] for i in range(2000)])
    assert np.all(th[:, 1] + th[:, 2] < 1)


# ---------------------------------------------------------- Euler-Maruyama ---

def test_gbm_moments_exact_for_em_chain():
    """theta2 = +inf turns the logistic step into X <- X(1 + a + c z): then
    E X_n = X0 (1+a)^n and E X_n^2 = X0^2 ((1+a)^2 + c^2)^n exactly for the
    discrete chain (independent, mean-0, variance-1 normals)."""
    dt = 0.01
    spec = W.logistic_spec(steps=100, t_end=1.0, n_obs=20, theta1=("point", 1.0, 0),
                           theta2=("point", math.inf, 0), theta3=("point", 0.5, 0))
    n = 60000
    sim = oracle.simulate(spec, 11, 0, n)
    a, c = 1.0 * dt, 0.5 * math.sqrt(dt)
    for k in range(20):
        steps = 5 * (k + 1)
        x = sim["summ"][:, k]
        assert _band(x, 10 * (1 + a) ** steps)
        assert _band(x**2, 100 * ((1 + a) ** 2 + c**2) ** steps)


def test_gbm_wrong_noise_scale_would_fail():
    """The second-moment band is tight enough to see a noise scale off by 10%."""
    dt = 0.01
    spec = W.logistic_spec(steps=100, t_end=1.0, n_obs=20, theta1=("point", 1.0, 0),
                           theta2=("point", math.inf, 0), theta3=("point", 0.5, 0))
    x = oracle.simulate(spec, 11, 0, 60000)["summ"][:, -1]
    a, c = 1.0 * dt, 0.55 * math.sqrt(dt)
    assert not _band(x**2, 100 * ((1 + a) ** 2 + c**2) ** 100)


def _logistic_ode(t, r, k, x0):
    e = math.exp(r * t)
    return k * x0 * e / (k + x0 * (e - 1))


def test_noise_free_logistic_converges_first_order_to_ode():
    """theta3 = 0: the EM chain is the explicit Euler method for the logistic
    ODE, whose solution is K X0 e^{rt} / (K + X0 (e^{rt} - 1)).  The error at
    the observation times is O(dt): it halves when dt halves."""
    r, k = 1.0, 100.0
    errs = []
    for steps in (1000, 2000, 4000, 8000):
        spec = W.logistic_spec(steps=steps, theta1=("point", r, 0), theta2=("point", k, 0),
                               theta3=("point", 0.0, 0))
        obs = oracle.simulate(spec, 1, 0, 1)["summ"][0]
        exact = np.array([_logistic_ode(0.5 * (j + 1), r, k, 10.0) for j in range(20)])
        errs.append(np.max(np.abs(obs - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.85 < q < 2.15 for q in ratios), (errs, ratios)
    assert errs[-1] < 0.02


def test_observation_times_and_absorption():
    """Observation k is X after step k*S/20; the full path agrees."""
    spec = W.logistic_spec(steps=200)
    for draw in range(5):
        th, _ = oracle.prior_draw(spec, 2, draw)
        path = oracle.logistic_path(spec, th, 2, draw)
        obs = oracle.simulate(spec, 2, draw, 1)["summ"][0]
        np.testing.assert_array_equal(obs, path[9::10])
        assert np.all(path >= 0)


def test_self_distance_is_zero():
    """Sampling with seed 0 at point priors equal to the observed theta
    reproduces the observed data: rho = 0 exactly."""
    with open(GOLDEN) as f:
        g = json.load(f)["logistic_S1000"]
    spec = W.logistic_point_spec(steps=1000)
    sim = oracle.simulate(spec, 0, 0, 1, y_obs=g["y_obs"])
    assert sim["dist"][0] == 0.0
    assert sim["stat"][0] == g["t_obs"]


# ---------------------------------------------------------- p-values ---

@pytest.mark.parametrize("prior_sd", [0.3, 1.0, 2.0])
def test_conjugate_normal_pvalue(prior_sd):
    """mu ~ N(0, l^2), y_j = mu + s z_j, T = ybar ~ N(0, l^2 + s^2/n):
    p = P(T >= t) = 1 - Phi(t / sqrt(l^2 + s^2/n))."""
    n_obs, sd, t_obs, n = 20, 1.0, 0.4, 200000
    spec = W.normal_mean_spec(n_obs=n_obs, noise_sd=sd, prior_sd=1.0)
    res = oracle.pvalue(spec, 0, "normal", [prior_sd], 21, 0, n, t_obs)
    p = 1 - stats.norm.cdf(t_obs / math.sqrt(prior_sd**2 + sd**2 / n_obs))
    assert abs(res["pvalue"][0] - p) <= 4 * math.sqrt(p * (1 - p) / n)
    assert res["count_ge"][0] == round(res["pvalue"][0] * n)


def test_pvalue_common_random_numbers_and_inclusive_tally():
    """Under lambda equal to the model's own prior, the tally equals a count
    over the per-draw statistics, with >= inclusive."""
    spec = W.pvalue_spec(steps=100)
    sim = oracle.simulate(spec, 1, 0, 3000)
    t_obs = float(np.sort(sim["stat"])[1500])  # an attained value: tests >=
    res = oracle.pvalue(spec, 0, "lognormal", [1.0, 0.5], 1, 0, 3000, t_obs)
    assert res["count_ge"][0] == int((sim["stat"] >= t_obs).sum())
    spec2 = W.pvalue_spec(steps=100)
    spec2["priors"][0] = ("lognormal", 0.0, 0.5)
    sim2 = oracle.simulate(spec2, 1, 0, 3000)
    assert res["count_ge"][1] == int((sim2["stat"] >= t_obs).sum())
    # CRN: theta2, theta3 and the path normals do not depend on lambda
    np.testing.assert_array_equal(sim["theta"][:, 1:], sim2["theta"][:, 1:])
    np.testing.assert_allclose(np.log(sim2["theta"][:, 0]), 0.5 * np.log(sim["theta"][:, 0]),
                               rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------- ABC ---

def test_top_count():
    assert oracle.top_count(0.01, 10000) == 100
    assert oracle.top_count(0.001, 100000) == 100
    assert oracle.top_count(0.01, 1) == 1
    assert oracle.top_count(0.01, 150) == 2
    assert oracle.top_count(1e-9, 5) == 1


def test_abc_top_fraction_and_fixed_agree_with_sorting():
    with open(GOLDEN) as f:
        y = np.array(json.load(f)["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=200)
    n = 2000
    sim = oracle.simulate(spec, 1, 500, n, y_obs=y)
    res = oracle.abc(spec, y, 1, 500, n, oracle.EPS_TOP_FRACTION, 0.02)
    k = oracle.top_count(0.02, n)
    order = np.lexsort((np.arange(n), sim["dist"]))[:k]
    np.testing.assert_array_equal(res["idx"], 500 + np.sort(order))
    assert res["eps_used"] == np.sort(sim["dist"])[k - 1]
    np.testing.assert_array_equal(res["dist"], sim["dist"][np.sort(order)])
    th = sim["theta"][np.sort(order)]
    np.testing.assert_allclose(res["mean"], th.mean(axis=0), rtol=1e-13)
    np.testing.assert_allclose(res["var"], th.var(axis=0, ddof=1), rtol=1e-11)
    # fixed eps at the same threshold accepts the same set (no ties here)
    fx = oracle.abc(spec, y, 1, 500, n, oracle.EPS_FIXED, res["eps_used"])
    np.testing.assert_array_equal(fx["idx"], res["idx"])
    # truncation keeps the true count
    tr = oracle.abc(spec, y, 1, 500, n, oracle.EPS_FIXED, res["eps_used"], capacity=5)
    assert tr["truncated"] and tr["n_accepted"] == k and len(tr["idx"]) == 5
    np.testing.assert_array_equal(tr["idx"], res["idx"][:5])


def test_abc_ties_broken_by_index():
    """With point priors and zero noise every draw has the same distance:
    the closest k are the k lowest indices."""
    spec = W.logistic_spec(steps=100, theta1=("point", 1, 0), theta2=("point", 100, 0),
                           theta3=("point", 0.0, 0))
    y = np.full(20, 50.0)
    res = oracle.abc(spec, y, 1, 10, 300, oracle.EPS_TOP_FRACTION, 0.05)
    np.testing.assert_array_equal(res["idx"], np.arange(10, 25))


# ---------------------------------------------------------- brute force ---

def _np_philox(ctr, key):
    c = [np.uint64(x) for x in ctr]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    m32 = np.uint64(0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(0x9E3779B9)) & m32
            k1 = (k1 + np.uint64(0xBB67AE85)) & m32
        p0 = np.uint64(0xD2511F53) * c[0]
        p1 = np.uint64(0xCD9E8D57) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & m32, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & m32]
    return [int(x) for x in c]


def _np_normals(seed, draw, count):
    # block b: three pairs; pair i has its radius from word i's top 23 bits
    # and its angle from word i's low 9 bits and 10 bits of word 3
    out = []
    for b in range((count + 5) // 6):
        w = _np_philox([b, 1, draw & 0xFFFFFFFF, draw >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        for i in range(3):
            u0 = (2 * (w[i] >> 9) + 1) / 2**24
            m = ((w[i] % 512) * 1024) + (w[3] // 2 ** (22 - 10 * i)) % 1024
            u1 = m / 2**19
            rad = math.sqrt(-2 * math.log(u0))
            out += [rad * math.cos(2 * math.pi * u1), rad * math.sin(2 * math.pi * u1)]
    return out[:count]


def test_tiny_brute_force_pipeline():
    """A separate loop-by-loop FP64 implementation on 48 draws, 20 steps,
    4 observations: theta, observations, distances, the accepted set."""
    spec = W.logistic_spec(steps=20, t_end=2.0, n_obs=4)
    seed, first, n = 17, 1000, 48
    y = np.array([10.5, 11.0, 12.0, 12.5])
    dt = 2.0 / 20
    bounds = [(0, 2), (50, 150), (0, 0.5)]
    ref_th, ref_obs = [], []
    for i in range(first, first + n):
        th = []
        for j, (lo, hi) in enumerate(bounds):
            w = _np_philox([j, 0, i & 0xFFFFFFFF, i >> 32], [seed & 0xFFFFFFFF, seed >> 32])
            th.append(lo + (hi - lo) * (2 * (w[0] >> 9) + 1) / 2**24)
        z = _np_normals(seed, i, 20)
        x, obs = 10.0, []
        for s in range(20):
            x = max(0.0, x + x * (th[0] * dt - th[0] * dt / th[1] * x + th[2] * math.sqrt(dt) * z[s]))
            if (s + 1) % 5 == 0:
                obs.append(x)
        ref_th.append(th)
        ref_obs.append(obs)
    ref_th, ref_obs = np.array(ref_th), np.array(ref_obs)
    ref_d = np.sqrt(((ref_obs - y) ** 2).sum(axis=1))
    sim = oracle.simulate(spec, seed, first, n, y_obs=y)
    np.testing.assert_allclose(sim["theta"], ref_th, rtol=1e-15)
    np.testing.assert_allclose(sim["summ"], ref_obs, rtol=1e-12)
    np.testing.assert_allclose(sim["dist"], ref_d, rtol=1e-12)
    res = oracle.abc(spec, y, seed, first, n, oracle.EPS_TOP_FRACTION, 0.25)
    k = 12
    np.testing.assert_array_equal(res["idx"], first + np.sort(np.argsort(ref_d, kind="stable")[:k]))


# ---------------------------------------------------------- GARCH ---

def test_garch_summary_definitions_match_scipy():
    rng = np.random.default_rng(3)
    r = rng.standard_t(5, size=2000) * 0.01
    s = oracle.garch_summaries(r)
    assert math.isclose(s[0], r.mean(), rel_tol=1e-12)
    assert math.isclose(s[1], r.var(), rel_tol=1e-12)
    assert math.isclose(s[2], stats.skew(r, bias=True), rel_tol=1e-10)
    assert math.isclose(s[3], stats.kurtosis(r, fisher=False, bias=True), rel_tol=1e-10)
    a = r**2 - (r**2).mean()
    full = np.correlate(a, a, mode="full")[len(a) - 1:]
    np.testing.assert_allclose(s[4:], full[1:11] / full[0], rtol=1e-10)


def test_garch_iid_special_case():
    """alpha = beta = 0: r_t = sqrt(omega) z_t exactly, so the series is the
    path normals scaled, and the summaries are those of i.i.d. N(0, omega)."""
    om = 4e-5
    spec = W.garch_spec(series_len=2000, omega=("point", om, 0), alpha=("point", 0.0, 0),
                        beta=("point", 0.0, 0), constraint=None)
    r = oracle.garch_series(spec, [om, 0.0, 0.0], 5, 3)
    z = np.array(_np_normals(5, 3, 2000))
    np.testing.assert_allclose(r, math.sqrt(om) * z, rtol=1e-13)
    sim = oracle.simulate(spec, 5, 0, 400)
    s = sim["summ"]
    assert _band(s[:, 0], 0.0)
    assert _band(s[:, 1], om * (1 - 1 / 2000))
    assert _band(s[:, 2], 0.0)
    assert abs(s[:, 3].mean() - 3.0) < 0.02
    for k in range(10):
        assert abs(s[:, 4 + k].mean()) < 4 * s[:, 4 + k].std() / math.sqrt(400) + 2e-3


def test_garch_stationary_variance_and_recursion():
    """Started at sigma2 = omega/(1-alpha-beta), E r_t^2 = omega/(1-alpha-beta)
    at every t; with alpha = 0 the variance never moves."""
    om, al, be = 1e-5, 0.1, 0.8
    spec = W.garch_spec(series_len=200, omega=("point", om, 0), alpha=("point", al, 0),
                        beta=("point", be, 0), constraint=None)
    rs = np.array([oracle.garch_series(spec, [om, al, be], 9, d) for d in range(20000)])
    sbar = om / (1 - al - be)
    for t in (0, 1, 5, 50, 199):
        assert _band(rs[:, t] ** 2, sbar)
    spec0 = W.garch_spec(series_len=50, omega=("point", om, 0), alpha=("point", 0.0, 0),
                         beta=("point", be, 0), constraint=None)
    r0 = oracle.garch_series(spec0, [om, 0.0, be], 9, 1)
    np.testing.assert_allclose(r0, math.sqrt(om / (1 - be)) * np.array(_np_normals(9, 1, 50)),
                               rtol=1e-13)


def test_garch_lag1_acf_textbook_form():
    """Loose check against the stationary lag-1 autocorrelation of r^2,
    alpha(1 - alpha beta - beta^2)/(1 - 2 alpha beta - beta^2) (finite-sample
    bias allowed for)."""
    om, al, be = 1e-5, 0.1, 0.6
    spec = W.garch_spec(series_len=2000, omega=("point", om, 0), alpha=("point", al, 0),
                        beta=("point", be, 0), constraint=None)
    s = oracle.simulate(spec, 13, 0, 300)["summ"]
    rho1 = al * (1 - al * be - be**2) / (1 - 2 * al * be - be**2)
    assert abs(s[:, 4].mean() - rho1) < 0.01
    rho2 = rho1 * (al + be)
    assert abs(s[:, 5].mean() - rho2) < 0.01


def test_garch_bar_scales_closed_form_and_bounds():
    """The error-bar scales: each is at least |summary| (triangle inequality),
    and for i.i.d. N(0, omega) returns (alpha = beta = 0) the mean's scale is
    sqrt(omega) E|z| = sqrt(2 omega / pi) and the skewness's is
    E|z|^3 = 2 sqrt(2 / pi)."""
    spec = W.garch_spec()
    sc = oracle.garch_bar_scales(spec, 1, range(200))
    s = oracle.simulate(spec, 1, 0, 200)["summ"]
    assert np.all(sc[:, :4] >= np.abs(s[:, :4]) * (1 - 1e-12))
    np.testing.assert_array_equal(sc[:, 1], np.abs(s[:, 1]))
    np.testing.assert_array_equal(sc[:, 3], np.abs(s[:, 3]))
    assert np.all(sc[:, 4:] == 1.0)
    om = 4e-5
    iid = W.garch_spec(series_len=2000, omega=("point", om, 0), alpha=("point", 0.0, 0),
                       beta=("point", 0.0, 0), constraint=None)
    si = oracle.garch_bar_scales(iid, 5, range(300))
    assert _band(si[:, 0], math.sqrt(2 * om / math.pi))
    assert _band(si[:, 2], 2 * math.sqrt(2 / math.pi))
