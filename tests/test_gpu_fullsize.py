"""Parity at the full workload sizes, in the launch configuration the benchmark
times (the autotuned shape; every shape gives identical results), on outputs
the oracle can compute one by one or in full where it finishes in seconds."""
import math

import numpy as np
import pytest

import oracle
import pps_workloads as W
from gpu_helpers import observed, rel_err, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    spec = W.logistic_spec(steps=1000)
    P.pps_autotune(spec, 1 << 21, use_cache=True)
    return P


def test_abc_n1e7_fixed_eps(P, torch):
    """N = 1e7, eps = the oracle pilot's 0.1 % quantile on [0, 1e5)."""
    g = observed()
    y = np.array(g["logistic_S1000"]["y_obs"])
    eps = g["abc_n1e7_pilot"]["eps"]
    spec = W.logistic_spec(steps=1000)
    n = 10_000_000
    cap = 20_000
    r = P.abc(spec, y, W.SAMPLING_SEED, 0, n, P.PPS_EPS_FIXED, eps, capacity=cap)
    assert r["status"] == P.PPS_OK
    idx = r["idx"].cpu().numpy().astype(np.int64)
    dist = r["dist"].cpu().numpy()
    theta = r["theta"].cpu().numpy()
    assert len(idx) == r["n_accepted"] and np.all(np.diff(idx) > 0)
    # (1) the pilot subsample: the accept set on [0, 1e5) is the oracle's
    pilot = oracle.abc(spec, y, W.SAMPLING_SEED, 0, 100_000, oracle.EPS_TOP_FRACTION, 0.001)
    sim = oracle.simulate(spec, W.SAMPLING_SEED, 0, 100_000, y_obs=y)
    band = set(np.nonzero(np.abs(sim["dist"] - eps) <= TOL * eps)[0].tolist())
    got = set(idx[idx < 100_000].tolist())
    assert got ^ set(pilot["idx"].tolist()) <= band
    # (2) sampled draws elsewhere, one by one: accepted ones within eps,
    # rejected ones beyond it (up to the band)
    rng = np.random.default_rng(0)
    acc = rng.choice(idx[idx >= 100_000], size=200, replace=False)
    pos = np.searchsorted(idx, acc)
    for i, p in zip(acc, pos):
        o = oracle.simulate(spec, W.SAMPLING_SEED, int(i), 1, y_obs=y)
        assert o["dist"][0] <= eps * (1 + TOL)
        assert abs(dist[p] - o["dist"][0]) <= TOL * o["dist"][0]
        np.testing.assert_array_equal(theta[:, p], o["theta"][0].astype(np.float32))
    acc_set = set(idx.tolist())
    rej = [int(i) for i in rng.integers(100_000, n, size=400) if int(i) not in acc_set][:200]
    for i in rej:
        o = oracle.simulate(spec, W.SAMPLING_SEED, i, 1, y_obs=y)
        assert o["dist"][0] > eps * (1 - TOL)
    # (3) FP64 posterior moments of the accepted theta (oracle prior draws)
    th64 = np.array([oracle.prior_draw(spec, W.SAMPLING_SEED, int(i))[0] for i in idx])
    np.testing.assert_allclose(r["mean"][:3], th64.mean(axis=0), rtol=1e-12)
    np.testing.assert_allclose(r["var"][:3], th64.var(axis=0, ddof=1), rtol=1e-10)


def test_abc_n1e7_top_fraction(P, torch):
    """Closest 0.1 % of 1e7: k = 10000 records; eps_used is the k-th
    smallest distance and every record lies within it."""
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=1000)
    r = P.abc(spec, y, W.SAMPLING_SEED, 0, 10_000_000, P.PPS_EPS_TOP_FRACTION, 0.001)
    assert r["n_accepted"] == 10_000
    d = r["dist"].cpu().numpy()
    assert d.max() == np.float32(r["eps_used"])
    rng = np.random.default_rng(1)
    idx = r["idx"].cpu().numpy().astype(np.int64)
    for p in rng.choice(len(idx), size=50, replace=False):
        o = oracle.simulate(spec, W.SAMPLING_SEED, int(idx[p]), 1, y_obs=y)
        assert abs(d[p] - o["dist"][0]) <= TOL * o["dist"][0]


@pytest.mark.parametrize("k", [0, 40, 63])
def test_pvalue_64x1e6(P, torch, k):
    """The 64-lambda batch at 1e6 draws per lambda against the full oracle run
    for three lambda values, draw by draw: the per-draw statistic of the same
    lambda row (the one-row kernel) decides every draw whose EM map contracts
    (th1 dt < 2) as the oracle does; the batch's count equals the number of
    those decisions, so it differs from the oracle's count by at most the
    number of chaotic draws whose decision flipped."""
    spec = W.pvalue_spec(steps=1000)
    t_obs = observed()["logistic_S1000"]["t_obs"]
    lam = W.lambda_grid(64)
    n = 1_000_000
    counts, p = P.prior_pred_pvalue(spec, 0, P.PPS_LOGNORMAL, lam, P.make_sampling(n, 0, 1), t_obs)
    ref = oracle.pvalue(spec, 0, "lognormal", [lam[k]], 1, 0, n, t_obs)
    sk = dict(spec, priors=[("lognormal", 0.0, float(lam[k]))] + spec["priors"][1:])
    o = oracle.simulate(sk, 1, 0, n)
    g = P.simulate(sk, 1, 0, n)
    dec_o = o["stat"] >= t_obs
    dec_g = g["stat"].cpu().numpy().astype(np.float64) >= t_obs
    chaotic = o["theta"][:, 0] * spec["t_end"] / spec["steps"] >= 2.0
    flips = int((dec_o != dec_g).sum())
    diff = abs(int(counts[k]) - int(ref["count_ge"][0]))
    print(f"lambda {lam[k]:.4f}: gpu {counts[k]} oracle {ref['count_ge'][0]} diff {diff}; "
          f"chaotic draws {int(chaotic.sum())}, decisions flipped {flips}")
    assert int(dec_o.sum()) == int(ref["count_ge"][0])
    assert np.array_equal(dec_o[~chaotic], dec_g[~chaotic])
    assert int(dec_g.sum()) == int(counts[k])
    assert diff <= flips
    if lam[k] <= 1.0:
        assert flips == 0 and diff == 0
    assert p[k] == counts[k] / n


def test_garch_n1e6_sampled(P, torch):
    """1e6 GARCH series: 300 sampled draws against the oracle's two-pass
    summaries, every summary within the 1e-5 bar."""
    from test_gpu_parity import GARCH_TOL, garch_errors, garch_scales
    spec = W.garch_spec()
    n = 1_000_000
    g = P.simulate(spec, W.SAMPLING_SEED, 0, n)
    summ = g["summ"].cpu().numpy()
    th = g["theta"].cpu().numpy()
    rng = np.random.default_rng(2)
    pick = np.sort(rng.choice(n, size=300, replace=False))
    o = np.array([oracle.simulate(spec, W.SAMPLING_SEED, int(i), 1)["summ"][0] for i in pick])
    ot = np.array([oracle.simulate(spec, W.SAMPLING_SEED, int(i), 1)["theta"][0] for i in pick[:20]])
    np.testing.assert_array_equal(th[:, pick[:20]].T, ot.astype(np.float32))
    errs = garch_errors(summ[:, pick].T.astype(np.float64), o, garch_scales(spec, W.SAMPLING_SEED, pick))
    for key, e in errs.items():
        print(f"GARCH 1e6 {key}: max {e.max():.2e} median {np.median(e):.2e}")
        assert e.max() <= GARCH_TOL, key
