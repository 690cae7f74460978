"""Parity of the BEGE log-likelihood (Sec. 4.2) with the FP64 oracle, through
the C ABI.

Bar.  Both sides compute the same discretised distribution functions in FP64
but not in the same way: the oracle sums F(u + h) and F(u - h) separately and
subtracts; the device accumulates the differences of the tails directly, each
one the Gamma(n, 1) mass of a short interval (a Taylor series about its
midpoint, or the difference of two upper functions Q in the upper tail),
forms most increments of P(p, .) between nodes as the integral of the
density's Taylor series over the interval (the rest by division-free
recurrences for P and Q), and uses different log/exp/lgamma
implementations.

* Where the oracle's FP64 difference exceeds 2^-26 it is its result.  The
  leading factor exp(a ln x - x - ln Gamma(a)) of P carries an absolute
  error of a few ulps of its largest term, and the oracle's two sums up to
  N_omega ulps each, so the numerators F(u + h) - F(u - h) = 2h f may differ
  by

      tol_F = 2^-45 (1 + a (1 + |ln a|)),   a = max(p_{t-1}, n_{t-1}) + N_omega / 100,

  and the log density by tol_F / (2h f) (at most ~1e-6 above 2^-26).
* Below 2^-26 the oracle evaluates the same difference in quad precision,
  exact to far beyond FP64, so the bar is the device's own error, relative:
  its interval masses are formed without cancellation (Taylor terms of one
  sign, or Q values of e^-y size each with its relative accuracy, differing
  by at least d |L_1| ~ 1e-4 of themselves), 1e-10, plus the rounding of
  their leading factor's exponent, which reaches a (1 + |ln a|) in size:
  tol_F read as a relative bound (1e-7 at the largest shapes of the tests);
  plus the FP64 rounding of the node positions, which the quad oracle does
  not have: w^0 + j dw cancels terms of size p s_p, so a node is up to
  8 ulp(2 p s_p + |u| + n s_n) off, which acts on the density as a shift of
  u by as much, |d ln f / du| times that (|d ln f / du| from the quad oracle
  by a central difference; it is large where a node's interval of the
  negative shock's law ends just above 0).
* Steps with non-positive shapes or scales are -inf on both sides exactly.
  A density below the smallest normal FP64 number (log f < -708.4) is
  outside what an FP64 evaluation resolves (the device's products underflow
  to denormals or 0, the oracle's quad value rounds to a denormal or 0):
  there both sides must lie below that level, and the vector's log L is not
  compared.  Every other step is finite on both sides, and log L is compared
  on every other vector within the sum of its steps' bars.
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


QUAD_BELOW = 2.0 ** -26   # the oracle's switch to its quad-precision difference
DEVICE_REL = 1e-10        # the device's relative bar where the oracle is exact
LOG_DBL_MIN = math.log(np.finfo(np.float64).tiny)  # -708.40: below, FP64 loses the density


def compare(P, thetas, r, n_omega=100, label=""):
    g = P.pps_bege_loglik(thetas, r, n_omega=n_omega, with_logdens=True)
    gll, gld = g["loglik"].cpu().numpy(), g["logdens"].cpu().numpy()
    worst_f, worst_q, n_quad, checked, n_low = 0.0, 0.0, 0, 0, 0
    oll, old_ = oracle.bege_loglik_batch(thetas, r, n_omega, with_logdens=True)
    for k, th in enumerate(thetas):
        o = {"loglik": oll[k], "logdens": old_[k]}
        ps, ns = shapes(th, r)
        valid = (ps > 0) & (ns > 0) & (th[1] > 0) & (th[6] > 0)
        # structurally -inf steps agree exactly
        assert np.all(gld[k][~valid] == -np.inf) and np.all(o["logdens"][~valid] == -np.inf)
        # densities below the smallest normal FP64 number: the device's
        # products underflow to denormals or 0 there, the oracle's quad value
        # rounds to a denormal or 0; both must lie below it (with a margin
        # of e^2 for a step that sits at the edge on one side only)
        low = valid & ((o["logdens"] < LOG_DBL_MIN) | (gld[k] < LOG_DBL_MIN))
        assert np.all(np.maximum(o["logdens"][low], gld[k][low]) < LOG_DBL_MIN + 2.0), (label, k)
        n_low += int(low.sum())
        valid = valid & ~low
        assert np.all(np.isfinite(gld[k][valid]) & np.isfinite(o["logdens"][valid])), (label, k)
        with np.errstate(invalid="ignore"):
            h2 = 2e-3 * np.sqrt(th[1] ** 2 * np.where(valid, ps, 0) + th[6] ** 2 * np.where(valid, ns, 0))
        a = np.maximum(ps, ns) + n_omega / 100.0
        tol_f = 2.0 ** -45 * (1.0 + a * (1.0 + np.abs(np.log(np.maximum(a, 1e-300)))))
        num_o = h2 * np.exp(o["logdens"])          # 2h f of the oracle (0 where -inf)
        num_g = h2 * np.exp(gld[k])
        fin = valid & np.isfinite(o["logdens"])
        quad = fin & (num_o <= QUAD_BELOW)
        fp = fin & ~quad
        n_quad += int(quad.sum())
        dif = np.abs(num_g - num_o)
        assert not (dif[fp] > tol_f[fp]).any(), (label, k, np.nonzero(fp)[0][dif[fp] > tol_f[fp]][:5])
        # where the oracle is exact: the device's relative error, its masses'
        # own (DEVICE_REL) plus their leading factor's exponent of size up to
        # a (1 + |ln a|), rounded to a few ulps (tol_F's factor, relative)
        # plus the FP64 rounding of the node positions: w^0 + j dw cancels
        # terms of size p s_p, so a node sits up to dw_err = 8 ulp(2 p s_p +
        # |u| + n s_n) off, which moves the density like a shift of u by as
        # much (large where a node's interval of the negative shock's law ends
        # just above 0): |d ln f / du| from the quad oracle, times dw_err
        rel_q = DEVICE_REL + tol_f
        u_all = r[1:] - th[10]
        for t in np.nonzero(quad)[0]:
            args = (ps[t], ns[t], th[1], th[6], n_omega)
            eta = 1e-7 * h2[t]
            fp_, fm_ = (oracle.bege_density_q(u_all[t] + sgn * eta, *args) for sgn in (1.0, -1.0))
            if fp_ > 0.0 and fm_ > 0.0:
                kappa = abs(math.log(fp_) - math.log(fm_)) / (2.0 * eta)
                dw_err = 8.0 * 2.0 ** -52 * (2.0 * ps[t] * th[1] + abs(u_all[t]) + ns[t] * th[6])
                rel_q[t] += kappa * dw_err
        assert not (dif[quad] > rel_q[quad] * num_o[quad]).any(), \
            (label, k, np.nonzero(quad)[0][dif[quad] > rel_q[quad] * num_o[quad]][:5])
        if fp.any():
            worst_f = max(worst_f, float((dif[fp] / tol_f[fp]).max()))
        if quad.any():
            worst_q = max(worst_q, float((dif[quad] / (rel_q[quad] * num_o[quad])).max()))
        if low.any():
            pass  # log L holds a density below the FP64 range: not compared
        elif np.isfinite(o["loglik"]):
            tol_ll = float(np.sum(tol_f[fp] / num_o[fp]) + np.sum(rel_q[quad])) + 1e-12 * abs(o["loglik"])
            assert abs(gll[k] - o["loglik"]) <= tol_ll, (label, k, gll[k], o["loglik"], tol_ll)
            checked += 1
        else:
            assert gll[k] == -np.inf
    print(f"{label}: {len(thetas)} vectors, {checked} finite log L compared, worst |dF|/tol_F "
          f"{worst_f:.3g}, {n_quad} steps against the quad difference (worst relative / bar {worst_q:.3g}), "
          f"{n_low} steps below the FP64 range")
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
    Every vector against the oracle (every step), and the device's own
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
    # every vector, every step (the oracle resolves the deep tails by its
    # quad-precision difference)
    gll, _ = compare(P, th, series, label="full batch")
    np.testing.assert_array_equal(gll, la)


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
