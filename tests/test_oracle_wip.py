"""Pins of the oracle's weak-informativity test (Sec. 4.1: Alg. 2, the SMC
evidence estimator of Alg. 3, the dose-response model of Eq. bioassay)
against facts fixed outside its code:

* the log-likelihood equals scipy's binomial log-pmf with the paper's link;
* the data generator: at lambda -> 0 the counts are Binomial(5, 1/2); under
  the base prior E y_i = n_i / 2 by symmetry and Var y_i has a closed form
  through E[p^2] (1-D quadrature); deaths fall as b0 + b1 x rises;
* the SMC evidence: the mean of independent estimates of p(D | lambda) equals
  the evidence computed by 2-D quadrature (the estimator is unbiased for Z),
  within its Monte Carlo error; the tempering schedule ends at 1 and the move
  counts follow ceil(ln c / ln(1 - p_acc));
* multinomial resampling: every ancestor is the categorical inverse
  distribution function of the float weights, in rational arithmetic;
* Alg. 2's p-values and alpha cut-offs equal numpy's counts and inverse-CDF
  quantiles of the returned evidences.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
import pps_workloads as W

SPEC = W.BIOASSAY
LAM0 = np.array(W.WIP_LAMBDA0)


def exact_log_evidence(y, lam, step=0.05):
    """log of the integral of L(b0, b1) N(b0; 0, l1^2) N(b1; 0, l2^2) on a dense
    grid (trapezoid rule; the integrand is smooth and decays like a Gaussian).
    The likelihood is written with scipy's log-sigmoid and log-gamma."""
    g0 = np.arange(-9.0 * lam[0], 9.0 * lam[0] + step, min(step, lam[0] / 50.0))
    g1 = np.arange(-9.0 * lam[1], 9.0 * lam[1] + step, min(step, lam[1] / 50.0))
    b0, b1 = np.meshgrid(g0, g1, indexing="ij")
    ll = np.zeros_like(b0)
    for n, x, k in zip(SPEC["n_trials"], SPEC["dose"], y):
        eta = b0 + b1 * x
        # p = 1 / (1 + e^eta): log p = log_expit(-eta), log(1 - p) = log_expit(eta)
        ll += (special.gammaln(n + 1) - special.gammaln(k + 1) - special.gammaln(n - k + 1)
               + k * special.log_expit(-eta) + (n - k) * special.log_expit(eta))
    lp = stats.norm.logpdf(b0, scale=lam[0]) + stats.norm.logpdf(b1, scale=lam[1])
    f = ll + lp
    m = f.max()
    z = integrate.trapezoid(integrate.trapezoid(np.exp(f - m), g1, axis=1), g0)
    return m + math.log(z)


def test_loglik_is_binomial_logpmf():
    rng = np.random.default_rng(0)
    for _ in range(50):
        y = rng.integers(0, 6, size=4)
        b0, b1 = rng.normal(0, 5), rng.normal(0, 3)
        ref = sum(stats.binom.logpmf(k, n, 1.0 / (1.0 + math.exp(b0 + b1 * x)))
                  for n, x, k in zip(SPEC["n_trials"], SPEC["dose"], y))
        assert abs(oracle.bio_loglik(SPEC, y, b0, b1) - ref) < 1e-10 * max(1.0, abs(ref))
    lam = np.array([2.0, 3.0])
    assert abs(oracle.bio_logprior(lam, 0.5, -1.0)
               - stats.norm.logpdf(0.5, scale=2.0) - stats.norm.logpdf(-1.0, scale=3.0)) < 1e-12


def test_data_at_a_point_prior_are_binomial_half():
    lam = np.array([1e-12, 1e-12])
    ys = np.array([oracle.bio_simulate(SPEC, lam, 3, i, oracle.P_DATA_BASE)[0] for i in range(8000)])
    counts = np.bincount(ys.ravel(), minlength=6)
    expected = stats.binom.pmf(np.arange(6), 5, 0.5) * ys.size
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < stats.chi2.ppf(0.999, 5)


def test_data_under_the_base_prior():
    n_sets = 20000
    out = [oracle.bio_simulate(SPEC, LAM0, 5, i, oracle.P_DATA_BASE) for i in range(n_sets)]
    ys = np.array([o[0] for o in out], np.float64)
    th = np.array([o[1] for o in out])
    np.testing.assert_allclose(th.std(axis=0), LAM0, rtol=0.03)
    for i, (n, x) in enumerate(zip(SPEC["n_trials"], SPEC["dose"])):
        s = math.hypot(LAM0[0], LAM0[1] * x)
        ep2 = integrate.quad(lambda e: (1.0 / (1.0 + math.exp(e))) ** 2 * stats.norm.pdf(e, scale=s),
                             -12 * s, 12 * s, limit=200)[0]
        var = n / 2.0 + n * (n - 1) * ep2 - n * n / 4.0
        assert abs(ys[:, i].mean() - n / 2.0) < 5.0 * math.sqrt(var / n_sets)
        assert abs(ys[:, i].var() / var - 1.0) < 0.04
        # deaths fall as the linear predictor rises
        eta = th[:, 0] + th[:, 1] * x
        assert np.corrcoef(ys[:, i], eta)[0, 1] < -0.5


@pytest.mark.parametrize("y,lam", [([0, 0, 0, 0], (10.0, 2.5)), ([1, 3, 4, 2], (10.0, 2.5)),
                                   ([5, 2, 0, 5], (3.0, 15.0)), ([2, 3, 2, 3], (0.5, 1.0))])
def test_smc_evidence_matches_quadrature(y, lam):
    lam = np.array(lam)
    exact = exact_log_evidence(y, lam)
    assert abs(exact - exact_log_evidence(y, lam, step=0.025)) < 1e-6  # grid converged
    cfg = dict(W.SMC_CONFIG)
    cfg["n_particles"] = 200
    reps = 60
    lz = np.array([oracle.smc_log_evidence(SPEC, y, lam, cfg, 17, r)["log_z"] for r in range(reps)])
    ratio = np.exp(lz - exact)
    err = ratio.std(ddof=1) / math.sqrt(reps)
    assert abs(ratio.mean() - 1.0) < 4.0 * err + 1e-3, (ratio.mean(), err)
    assert ratio.std() < 0.5  # the estimator is not degenerate


def test_smc_temper_meets_the_ess_condition():
    rng = np.random.default_rng(3)
    cfg = W.SMC_CONFIG
    for trial in range(20):
        ll = rng.normal(-10.0, rng.uniform(0.5, 30.0), size=500)
        t = float(rng.uniform(0.0, 0.9))
        d = oracle.smc_temper(ll, t, 1, cfg)

        def ess(delta):
            w = np.exp(delta * (ll - ll.max()))
            return w.sum() ** 2 / (w * w).sum()
        rest = 1.0 - t
        if d == rest:
            assert ess(rest) >= 250.0
        else:
            # the root of ESS = N_p / 2, approached from the ESS >= N_p / 2 side
            assert 250.0 - 1e-9 <= ess(d) < 250.0 + 1e-6
            assert ess(d + 1e-6 * rest) < 250.0
    # the step cap takes the whole remaining increment
    ll = np.linspace(-500.0, 0.0, 500)
    assert oracle.smc_temper(ll, 0.25, cfg["max_steps"], cfg) == 0.75


def test_smc_resampling_is_inversion_of_the_weights():
    rng = np.random.default_rng(5)
    w = rng.uniform(0.0, 1.0, size=300)
    w[rng.integers(0, 300, size=30)] = 0.0
    w[7] = 1.0
    anc = oracle.smc_resample(w, 3, 44, 6)
    q = np.floor(w * 2.0 ** 52).astype(np.uint64)
    cum = np.cumsum(q)
    words = np.array([oracle.stream_block(3, 44, 6, 0x60000000 + i) for i in range(300)], np.uint64)
    r64 = (words[:, 1] << np.uint64(32)) | words[:, 0]
    u = np.array([(int(r) * int(cum[-1])) >> 64 for r in r64], dtype=object)
    ref = [int(np.searchsorted(cum, np.uint64(x), side="right")) for x in u]
    np.testing.assert_array_equal(anc, ref)
    assert np.all(w[anc] > 0.0)
    # frequencies follow the weights over many steps
    counts = np.zeros(300)
    for step in range(1, 201):
        counts += np.bincount(oracle.smc_resample(w, 3, 44, step), minlength=300)
    expected = w / w.sum() * counts.sum()
    nz = expected > 0
    chi2 = ((counts[nz] - expected[nz]) ** 2 / expected[nz]).sum()
    assert chi2 < stats.chi2.ppf(0.999, nz.sum() - 1)


@pytest.mark.parametrize("case", ["uniform", "dyadic", "one_nonzero", "tiny_and_large"])
def test_smc_resampling_is_categorical_inversion(case):
    """Multinomial resampling is the inverse distribution function of the
    categorical law with probabilities w_i / sum w (Alg. 3, resampling step):
    with the uniform U = r / 2^64 of each particle's 64-bit random integer r,
    the ancestor is the first i whose exact cumulative share C_i = (w_1 + ...
    + w_i) / sum w exceeds U.  Checked in rational arithmetic on the float
    weights themselves, not on their fixed-point images, so the fixed-point
    reading is held to the textbook law: it may move an ancestor only for a
    uniform within (n + 2) 2^-52 / sum w of a boundary C_i (the truncation of
    each weight and the flooring of U), and none of these draws lands there."""
    from fractions import Fraction
    rng = np.random.default_rng({"uniform": 15, "dyadic": 16, "one_nonzero": 17, "tiny_and_large": 18}[case])
    n = 257
    if case == "uniform":
        w = rng.uniform(0.0, 1.0, size=n)
        w[rng.integers(0, n, size=40)] = 0.0
    elif case == "dyadic":
        w = rng.integers(0, 9, size=n) / 8.0
    elif case == "one_nonzero":
        w = np.zeros(n)
        w[123] = 0.3
    else:
        w = np.where(rng.uniform(size=n) < 0.5, 1e-300, 1.0) * rng.uniform(0.5, 1.0, size=n)
    step = 9
    anc = oracle.smc_resample(w, 5, 71, step)
    words = np.array([oracle.stream_block(5, 71, step, 0x60000000 + i) for i in range(n)], np.uint64)
    r64 = [(int(a) << 32) | int(b) for a, b in zip(words[:, 1], words[:, 0])]
    wq = [Fraction(float(x)) for x in w]
    tot = sum(wq)
    cum, acc = [], Fraction(0)
    for x in wq:
        acc += x
        cum.append(acc / tot)
    band = Fraction(n + 2, 2 ** 52) / tot
    for i, r in enumerate(r64):
        U = Fraction(r, 2 ** 64)
        exact = next(k for k, c in enumerate(cum) if c > U)
        near = min(abs(U - c) for c in cum)
        assert near > band, (case, i)
        assert anc[i] == exact, (case, i, anc[i], exact)
        assert w[anc[i]] > 0.0
    if case == "one_nonzero":
        assert np.all(anc == 123)


def test_smc_proposal_factor():
    rng = np.random.default_rng(6)
    b = rng.multivariate_normal([1.0, -2.0], [[4.0, 1.5], [1.5, 2.0]], size=400)
    l11, l21, l22 = oracle.smc_proposal(b[:, 0], b[:, 1], 1.7)
    ref = np.linalg.cholesky(1.7 ** 2 * np.cov(b.T, ddof=1))
    np.testing.assert_allclose([l11, l21, l22], [ref[0, 0], ref[1, 0], ref[1, 1]], rtol=1e-12)
    assert list(oracle.smc_proposal(np.ones(10), np.arange(10.0), 1.0)) == [0.0, 0.0, pytest.approx(np.std(np.arange(10.0), ddof=1))]


def test_smc_moves():
    cfg = W.SMC_CONFIG
    assert oracle.smc_moves(0, 500, cfg) == cfg["max_mcmc"]
    assert oracle.smc_moves(500, 500, cfg) == 1
    for acc in (1, 17, 150, 250, 499):
        p = acc / 500
        assert oracle.smc_moves(acc, 500, cfg) == min(max(math.ceil(math.log(0.01) / math.log(1 - p)), 1),
                                                      cfg["max_mcmc"])


def test_smc_schedule():
    y = np.array([1, 3, 4, 2])
    r = oracle.smc_log_evidence(SPEC, y, LAM0, W.SMC_CONFIG, 2, 9)
    tr = r["trace"]
    t, delta, pacc, moves = tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3]
    assert r["n_steps"] >= 2 and t[-1] == 1.0
    assert np.all(np.diff(t) > 0) and np.all(delta > 0)
    np.testing.assert_allclose(np.cumsum(delta)[:-1], t[:-1], rtol=1e-12)
    c = W.SMC_CONFIG["c"]
    for p, m in zip(pacc, moves):
        assert m == oracle.smc_moves(int(round(p * 500)), 500, W.SMC_CONFIG)
        if 0.0 < p < 1.0:
            assert m == min(max(math.ceil(math.log(c) / math.log(1.0 - p)), 1), W.SMC_CONFIG["max_mcmc"])


def test_wip_pvalues_and_cutoffs():
    lam = W.wip_lambdas(3, seed=4)
    cfg = dict(W.SMC_CONFIG)
    cfg["n_particles"] = 100
    n = 40
    r = oracle.wip_test(SPEC, lam, n, cfg, 8, 0.1)
    for k in range(lam.shape[0]):
        zk = np.sort(r["log_zk"][k])
        p = np.searchsorted(zk, r["log_z0"][k], side="right") / n
        np.testing.assert_array_equal(r["pvalues"][k], p)
        assert r["gamma"][k] == np.quantile(p, 0.1, method="inverted_cdf")
    # the evidences are those of single runs with the documented indices
    y0, _ = oracle.bio_simulate(SPEC, lam[0], 8, 3, oracle.P_DATA_BASE)
    one = oracle.smc_log_evidence(SPEC, y0, lam[2], cfg, 8, (2 * n + 3) * 2)
    assert one["log_z"] == r["log_z0"][2, 3]
    yk, _ = oracle.bio_simulate(SPEC, lam[2], 8, 2 * n + 5, oracle.P_DATA_K)
    one = oracle.smc_log_evidence(SPEC, yk, lam[2], cfg, 8, (2 * n + 5) * 2 + 1)
    assert one["log_z"] == r["log_zk"][2, 5]
