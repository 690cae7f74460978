"""Parity of the toggle-switch kernel (Sec. 3.2; one draw per workgroup, cells
across lanes, quantiles by an LDS sort) with the FP64 oracle, through the C ABI.

Bars (FP32 simulation vs FP64 oracle on the same random numbers):
* theta: the oracle's FP64 draw rounded to FP32, bit for bit;
* quantile summaries: relative error <= TSW_TOL each, and the median over all
  summaries <= TSW_MEDIAN.  A quantile is an order statistic, so it moves by at
  most the largest change of the cells near its rank; FP32 rounding of the
  levels (6e-8 per step, damped by the 0.97 decay) and of the hardware log2 /
  exp2 powers (up to ~1e-6 relative for beta log2 v ~ 70) give cell errors of
  1e-7 .. 1e-5, larger only for cells near the switch's separatrix, which
  rarely sit at a quantile's rank (measured: max 3e-6, median 4e-8);
* distance and statistic: relative TSW_TOL;
* ABC accept sets: identical except draws whose oracle distance lies within
  TSW_TOL * eps of eps;
* tallies: decisions may differ only for summaries within TSW_TOL of the
  observed value.
"""
import numpy as np
import pytest

import oracle
import pps_workloads as W
from gpu_helpers import observed, rel_err, require_gpu

pytestmark = pytest.mark.gpu

TSW_TOL = 2e-5
TSW_MEDIAN = 2e-7


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    return P


def check_draws(P, spec, g, o, y_obs=None, label=""):
    th = g["theta"].cpu().numpy().T
    np.testing.assert_array_equal(th, o["theta"].astype(np.float32))
    summ = g["summ"].cpu().numpy().T.astype(np.float64)
    e = rel_err(summ, o["summ"])
    print(f"{label} quantiles: max {e.max():.2e} median {np.median(e):.2e} p99 {np.quantile(e, 0.99):.2e}")
    assert e.max() <= TSW_TOL
    assert np.median(e) <= TSW_MEDIAN
    np.testing.assert_allclose(g["stat"].cpu().numpy(), o["stat"], rtol=TSW_TOL)
    if y_obs is not None:
        np.testing.assert_allclose(g["dist"].cpu().numpy(), o["dist"], rtol=TSW_TOL)


@pytest.mark.parametrize("n_cells,steps,n_q", [(1000, 599, 19), (777, 200, 19), (8192, 30, 64),
                                               (1, 15, 3), (64, 1, 19)])
def test_toggle_summaries(P, torch, n_cells, steps, n_q):
    spec = W.toggle_spec(n_cells=n_cells, steps=steps, n_quantiles=n_q)
    n = 24
    y_obs = np.linspace(200.0, 700.0, n_q)
    o = oracle.simulate(spec, W.SAMPLING_SEED, 5, n, y_obs=y_obs)
    g = P.simulate(spec, W.SAMPLING_SEED, 5, n, y_obs=y_obs)
    check_draws(P, spec, g, o, y_obs, f"C={n_cells} S={steps} K={n_q}")


def test_toggle_dt_not_one(P, torch):
    spec = W.toggle_spec(n_cells=600, steps=400, dt=0.25)
    o = oracle.simulate(spec, 9, 0, 16)
    g = P.simulate(spec, 9, 0, 16)
    check_draws(P, spec, g, o, None, "dt=0.25")


def test_toggle_launch_shapes_identical(P, torch):
    spec = W.toggle_spec(n_cells=1500, steps=100)
    keep = P.pps_get_launch_shape(P.CLASS_CELLS)
    outs = []
    try:
        for sh in P.CELL_SHAPES:
            P.pps_set_launch_shape(P.CLASS_CELLS, *sh)
            g = P.simulate(spec, 3, 100, 40, y_obs=np.full(19, 400.0))
            outs.append({k: v.cpu().numpy() for k, v in g.items()})
    finally:
        P.pps_set_launch_shape(P.CLASS_CELLS, *keep)
    for o in outs[1:]:
        for k in o:
            np.testing.assert_array_equal(o[k], outs[0][k])


def test_toggle_abc_top_fraction(P, torch):
    spec = W.toggle_spec(n_cells=400, steps=200)
    obs = oracle.simulate(W.toggle_point_spec(n_cells=400, steps=200), W.OBS_SEED, W.OBS_DRAW, 1)
    y = obs["summ"][0]
    n = 3000
    r = P.abc(spec, y, W.SAMPLING_SEED, 0, n, P.PPS_EPS_TOP_FRACTION, 0.02)
    ref = oracle.abc(spec, y, W.SAMPLING_SEED, 0, n, oracle.EPS_TOP_FRACTION, 0.02)
    assert r["n_accepted"] == ref["n_accepted"] == 60
    sim = oracle.simulate(spec, W.SAMPLING_SEED, 0, n, y_obs=y)
    eps = ref["eps_used"]
    band = set(np.nonzero(np.abs(sim["dist"] - eps) <= TSW_TOL * eps)[0].tolist())
    got = set(r["idx"].cpu().numpy().astype(np.int64).tolist())
    assert got ^ set(ref["idx"].astype(np.int64).tolist()) <= band
    assert abs(r["eps_used"] - eps) <= TSW_TOL * eps
    if got == set(ref["idx"].astype(np.int64).tolist()):
        np.testing.assert_allclose(r["mean"][:7], ref["mean"], rtol=1e-12)
        np.testing.assert_allclose(r["var"][:7], ref["var"], rtol=1e-10)
        th = r["theta"].cpu().numpy().T
        np.testing.assert_array_equal(th, ref["theta"].astype(np.float32))


def test_toggle_summary_tally_and_pvalue(P, torch):
    spec = W.toggle_spec(n_cells=300, steps=150)
    n = 1500
    obs = np.array(observed()["toggle_C8000_T600"]["y_obs"])
    counts = P.pps_summary_tally(spec, P.make_sampling(n, 0, 4), obs)
    ref = oracle.summary_tally(spec, 4, 0, n, obs)
    sim = oracle.simulate(spec, 4, 0, n)
    near = (np.abs(sim["summ"] - obs[None, :]) <= TSW_TOL * np.abs(obs[None, :])).sum(axis=0)
    assert np.all(np.abs(counts.astype(np.int64) - ref.astype(np.int64)) <= near)
    # p-values of the mean quantile over an upper bound of beta_u's prior
    t_obs = observed()["toggle_C8000_T600"]["t_obs"]
    lam = [1.0, 3.0, 7.0]
    c, p = P.prior_pred_pvalue(spec, 5, P.PPS_UNIFORM, lam, P.make_sampling(n, 0, 4), t_obs)
    ro = oracle.pvalue(spec, 5, "uniform", lam, 4, 0, n, t_obs)
    for k, l in enumerate(lam):
        sk = dict(spec)
        sk["priors"] = list(spec["priors"])
        sk["priors"][5] = ("uniform", 0.0, l)
        st = oracle.simulate(sk, 4, 0, n)["stat"]
        near = int((np.abs(st - t_obs) <= TSW_TOL * t_obs).sum())
        assert abs(int(c[k]) - int(ro["count_ge"][k])) <= near
        assert p[k] == c[k] / n


def test_toggle_full_size_sampled(P, torch):
    """C = 8000 cells, 599 steps, N = 8064 (the paper's prior-predictive run):
    two blocks of 8 consecutive draws at seeded offsets against the oracle."""
    spec = W.toggle_spec()
    y = np.array(observed()["toggle_C8000_T600"]["y_obs"])
    n = W.TOGGLE_PPS["n"]
    g = P.simulate(spec, W.SAMPLING_SEED, 0, n, y_obs=y)
    rng = np.random.default_rng(7)
    for start in rng.choice(n - 8, size=2, replace=False):
        o = oracle.simulate(spec, W.SAMPLING_SEED, int(start), 8, y_obs=y)
        sl = slice(int(start), int(start) + 8)
        gs = {k: v[..., sl] for k, v in g.items()}
        check_draws(P, spec, gs, o, y, f"full size draws {start}..")


def test_toggle_invalid(P, torch):
    spec = W.toggle_spec(n_cells=P.PPS_TSW_MAX_CELLS + 1)
    with pytest.raises(P.PPSError):
        P.simulate(spec, 1, 0, 4)
