"""Parity of the BEGE log-likelihood (Sec. 4.2) with the FP64 oracle, through
the C ABI.

Bar.  Both sides compute the same discretised distribution functions in FP64
but not in the same way: the oracle sums F(u + h) and F(u - h) separately and
subtracts; the device accumulates the differences of the tails directly, each
one the Gamma(n, 1) mass of a short interval (a Taylor series about its
midpoint, exact to rounding, where the oracle's two incomplete gamma values
cancel), evaluates P(a, x) by division-free recurrences, and uses different
log/exp/lgamma implementations.
The leading factor exp(a ln x - x - ln Gamma(a)) of P carries an absolute
error of a few ulps of its largest term, and the oracle's two sums carry up
to N_omega ulps each, so the numerator F(u + h) - F(u - h) = 2h f may differ
by

    tol_F = 2^-45 (1 + a (1 + |ln a|)),   a = max(p_{t-1}, n_{t-1}) + N_omega / 100,

and the log density by tol_F / (2h f).  A step whose oracle numerator is
itself below tol_F is not resolved by either side: there only "both are
small or -inf" is checked, and the log-likelihood of its vector is compared
only in that weak sense.  Steps with non-positive shapes are -inf on both
sides exactly.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import pps_workloads as W
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    return P


@pytest.fixture(scope="module")
def series():
    with open(os.path.join(HERE, "golden", "observed.json")) as f:
        return np.array(json.load(f)["bege_T1099"]["r"])


def shapes(th, r):
    """(p_{t-1}, n_{t-1}) for t = 1..T by Eq. shape (for the tolerances)."""
    p0, sp, rp, pp, pn, n0, sn, rn, np_, nn, mu = th
    T = len(r) - 1
    P_, N_ = np.empty(T), np.empty(T)
    p, n = p0, n0
    for t in range(1, T + 1):
        P_[t - 1], N_[t - 1] = p, n
        u = r[t] - mu
        p = p0 + rp * p + (pp if u >= 0 else pn) * u * u / (2 * sp * sp)
        n = n0 + rn * n + (np_ if u >= 0 else nn) * u * u / (2 * sn * sn)
    return P_, N_


def compare(P, thetas, r, n_omega=100, label=""):
    g = P.pps_bege_loglik(thetas, r, n_omega=n_omega, with_logdens=True)
    gll, gld = g["loglik"].cpu().numpy(), g["logdens"].cpu().numpy()
    worst, unresolved, checked = 0.0, 0, 0
    for k, th in enumerate(thetas):
        o = oracle.bege_loglik(th, r, n_omega)
        ps, ns = shapes(th, r)
        valid = (ps > 0) & (ns > 0) & (th[1] > 0) & (th[6] > 0)
        # structurally -inf steps agree exactly
        assert np.all(gld[k][~valid] == -np.inf) and np.all(o["logdens"][~valid] == -np.inf)
        with np.errstate(invalid="ignore"):
            h2 = 2e-3 * np.sqrt(th[1] ** 2 * np.where(valid, ps, 0) + th[6] ** 2 * np.where(valid, ns, 0))
        a = np.maximum(ps, ns) + n_omega / 100.0
        tol_f = 2.0 ** -45 * (1.0 + a * (1.0 + np.abs(np.log(np.maximum(a, 1e-300)))))
        num_o = h2 * np.exp(o["logdens"])          # 2h f of the oracle (0 where -inf)
        num_g = h2 * np.exp(gld[k])
        res = valid & (num_o > tol_f)
        bad = np.abs(num_g[res] - num_o[res]) > tol_f[res]
        assert not bad.any(), (label, k, np.nonzero(res)[0][bad][:5])
        if res.any():
            worst = max(worst, float((np.abs(num_g[res] - num_o[res]) / tol_f[res]).max()))
        # unresolved steps: both numerators below 2 tol_F (or -inf)
        un = valid & ~res
        unresolved += int(un.sum())
        assert np.all(num_g[un] <= 2.0 * tol_f[un])
        if not un.any() and valid.all():
            tol_ll = float(np.sum(tol_f / num_o)) + 1e-12 * abs(o["loglik"])
            assert abs(gll[k] - o["loglik"]) <= tol_ll, (label, k, gll[k], o["loglik"], tol_ll)
            checked += 1
        elif not valid.all():
            assert gll[k] == -np.inf and o["loglik"] == -np.inf
        # (a vector with an unresolved step is compared step by step only)
    print(f"{label}: {len(thetas)} vectors, {checked} log L compared, worst |dF|/tol {worst:.3g}, "
          f"{unresolved} unresolved steps")
    return gll, gld


def test_bege_prior_batch(P, torch, series):
    th = W.bege_prior_draws(192, seed=5)
    compare(P, th, series, label="prior draws, T=1099")


def test_bege_near_truth(P, torch, series):
    rng = np.random.default_rng(2)
    base = np.array(W.BEGE_THETA_OBS)
    th = base * (1.0 + 0.1 * rng.standard_normal((64, 11)))
    th[:, 8] = base[8] + 0.005 * rng.standard_normal(64)
    gll, _ = compare(P, th, series, label="near the generating theta")
    assert np.isfinite(gll).sum() >= 48


@pytest.mark.parametrize("T", [1, 2, 63, 64, 65, 130, 257])
def test_bege_ragged_lengths(P, torch, series, T):
    th = W.bege_prior_draws(24, seed=T)
    th[0] = W.BEGE_THETA_OBS
    compare(P, th, series[:T + 1], label=f"T={T}")


@pytest.mark.parametrize("n_omega", [2, 7, 100, 1000])
def test_bege_node_counts(P, torch, series, n_omega):
    th = W.bege_prior_draws(16, seed=100 + n_omega)
    th[0] = W.BEGE_THETA_OBS
    compare(P, th, series[:300], n_omega=n_omega, label=f"N_omega={n_omega}")


def test_bege_domain_edges(P, torch, series):
    base = np.array(W.BEGE_THETA_OBS)
    rows = [base.copy() for _ in range(6)]
    rows[0][1] = 0.0            # s_p = 0: outside the domain, every step -inf
    rows[1][6] = -0.01          # s_n < 0
    rows[2][8] = -0.2           # phi_n+ = -0.2: n_t turns negative after a large positive u
    rows[3][1] = 1e-4           # tiny s_p: huge shapes
    rows[4][6] = 1e-4           # tiny s_n: huge negative shapes
    rows[5][0] = 1e-4           # tiny p0
    th = np.array(rows)
    gll, gld = compare(P, th, series[:400], label="domain edges")
    assert gll[0] == -np.inf and np.all(gld[0] == -np.inf)
    assert gll[1] == -np.inf
    assert gll[2] == -np.inf and np.isfinite(gld[2][0])


def test_bege_full_batch_sampled(P, torch, series):
    """The benchmark batch: N_p = 1024 prior draws, T = 1099, N_omega = 100.
    16 sampled vectors against the oracle (every step), and the device's own
    repeatability (bit-identical results on a second call, with and without
    the per-step output)."""
    cfg = W.BEGE_BATCH
    th = W.bege_prior_draws(cfg["n_theta"], seed=cfg["seed"])
    a = P.pps_bege_loglik(th, series, n_omega=cfg["n_omega"], with_logdens=True)
    b = P.pps_bege_loglik(th, series, n_omega=cfg["n_omega"])
    la, lb = a["loglik"].cpu().numpy(), b["loglik"].cpu().numpy()
    np.testing.assert_array_equal(la, lb)
    ld = a["logdens"].cpu().numpy()
    # the sum of the per-step log densities (fixed order on the device)
    fin = np.isfinite(la)
    np.testing.assert_allclose(la[fin], ld[fin].sum(axis=1), rtol=1e-12)
    assert np.all(np.isneginf(ld[~fin]).any(axis=1))
    rng = np.random.default_rng(0)
    pick = rng.choice(cfg["n_theta"], size=16, replace=False)
    gll, _ = compare(P, th[pick], series, label="full batch, sampled")
    np.testing.assert_array_equal(gll, la[pick])


def test_bege_invalid(P, torch, series):
    with pytest.raises(P.PPSError):
        P.pps_bege_loglik(W.bege_prior_draws(2), series, n_omega=1)


def test_bege_count_ops(P, torch, series):
    """The counting instantiation reports the work of the same batch: more
    work for more nodes, none lost between calls, and results unchanged."""
    th = W.bege_prior_draws(32, seed=9)
    a = P.pps_bege_count_ops(th, series[:200], 100)
    b = P.pps_bege_count_ops(th, series[:200], 100)
    c = P.pps_bege_count_ops(th, series[:200], 200)
    assert a == b and a > 0 and c > 1.5 * a
    # at least the fixed work of every valid step: two lgammas and one log
    assert a > 32 * 199 * 0.5 * (2 * 200 + 90)
    ll = P.pps_bege_loglik(th, series[:200])["loglik"].cpu().numpy()
    ll2 = P.pps_bege_loglik(th, series[:200])["loglik"].cpu().numpy()
    np.testing.assert_array_equal(ll, ll2)
