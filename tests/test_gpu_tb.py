"""Parity of the tuberculosis Gillespie kernel (App. B; one run per 64-lane
workgroup, genotype counts in LDS) with the FP64 oracle, through the C ABI.

Bar.  Every decision of a run is integer arithmetic on the same random words
(the case number floor(w N / 2^32), the event type against thresholds that
both sides form with the same single FP64 operations, the lowest empty slot),
so event counts, status and the sampled genotype counts agree exactly, and the
summaries g/n_s and H = 1 - sum n_i^2 / n_s^2, formed in FP64 from those
integers, agree bit for bit before the device rounds them to FP32.  theta is
the oracle's FP64 draw rounded to FP32.  Distances (FP32 on the device)
agree to 1e-6 relative; ABC accept sets are identical up to draws within
that band of the cut.
"""
import numpy as np
import pytest

import oracle
import pps_workloads as W
from gpu_helpers import observed, require_gpu

pytestmark = pytest.mark.gpu

DIST_TOL = 1e-6


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    return P


def check(P, spec, seed, first, n, y_obs=None, label=""):
    o = oracle.tb_simulate(spec, seed, first, n)
    samp = P.make_sampling(n, first, seed)
    ev = P.pps_tb_events(spec, samp)
    np.testing.assert_array_equal(ev["status"].cpu().numpy(), o["status"])
    np.testing.assert_array_equal(ev["events"].cpu().numpy().astype(np.uint64), o["events"])
    g = P.simulate(spec, seed, first, n, y_obs=y_obs)
    np.testing.assert_array_equal(g["theta"].cpu().numpy().T, o["theta"].astype(np.float32))
    np.testing.assert_array_equal(g["summ"].cpu().numpy().T, o["summ"].astype(np.float32))
    np.testing.assert_array_equal(g["stat"].cpu().numpy(),
                                  (0.5 * (o["summ"][:, 0] + o["summ"][:, 1])).astype(np.float32))
    if y_obs is not None:
        d = np.sqrt(((o["summ"] - np.asarray(y_obs, np.float32).astype(np.float64)) ** 2).sum(axis=1))
        np.testing.assert_allclose(g["dist"].cpu().numpy(), d, rtol=DIST_TOL, atol=1e-7)
    st = np.bincount(o["status"], minlength=3)
    print(f"{label}: {n} draws, complete/extinct/truncated {st.tolist()}, events "
          f"median {np.median(o['events']):.0f} max {o['events'].max()}")
    return o


@pytest.mark.parametrize("n_stop,n_sample,max_events", [(200, 50, 1 << 20), (1000, 120, 1 << 20),
                                                        (777, 473, 1 << 20), (64, 100, 1 << 20),
                                                        (2500, 473, 4000), (65, 1024, 1 << 20)])
def test_tb_runs(P, torch, n_stop, n_sample, max_events):
    spec = W.tb_spec(n_stop=n_stop, n_sample=n_sample, max_events=max_events)
    check(P, spec, W.SAMPLING_SEED, 7, 96, y_obs=[0.5, 0.9],
          label=f"K={n_stop} n={n_sample} cap={max_events}")


def test_tb_edges(P, torch):
    # many initial cases, a start at the stop size (no events), the largest
    # population and sample, no constraint (subcritical draws die out)
    check(P, W.tb_spec(n_stop=300, n_sample=40, x0=37.0), 3, 0, 48, label="x0=37")
    o = check(P, W.tb_spec(n_stop=50, n_sample=20, x0=50.0), 3, 0, 8, label="x0=K")
    assert np.all(o["events"] == 0)
    check(P, W.tb_spec(n_stop=W.TB_PPS["n_stop"] * 0 + 16384, n_sample=1024, max_events=1 << 18), 5, 0,
          6, label="K=16384 n=1024")
    nc = W.tb_spec(n_stop=400, n_sample=60)
    nc["constraint"] = None
    o = check(P, nc, 8, 0, 64, label="no constraint")
    assert (o["status"] == oracle.TB_EXTINCT).sum() > 16


@pytest.mark.parametrize("n_stop,max_events,x0", [(2, 1 << 20, 1.0), (3, 1 << 20, 1.0), (200, 1, 1.0),
                                                  (200, 127, 1.0), (200, 129, 5.0), (400, 255, 1.0),
                                                  (500, 4001, 1.0), (300, 1 << 20, 299.0)])
def test_tb_stop_test_edges(P, torch, n_stop, max_events, x0):
    # the kernel tests the stop rule once per stretch of events that cannot
    # end the run (the count moves by one per event): stop sizes of 2 and 3
    # and a start one case below the stop size make every stretch one event
    # long; odd caps and caps inside a 64-event half end a run mid-stretch
    spec = W.tb_spec(n_stop=n_stop, n_sample=min(40, n_stop), max_events=max_events, x0=x0)
    o = check(P, spec, W.SAMPLING_SEED, 11, 48, y_obs=[0.5, 0.9],
              label=f"K={n_stop} cap={max_events} x0={x0:g}")
    assert np.all(o["events"] <= max_events)
    if max_events < 1 << 20:
        assert np.any(o["status"] == oracle.TB_TRUNCATED)


def test_tb_point_prior_reproduces_the_observed_summaries(P, torch):
    g = observed()["tb_K10000_n473"]
    spec = W.tb_point_spec(tuple(g["theta"]), n_stop=g["n_stop"], n_sample=g["n_sample"])
    out = P.simulate(spec, g["seed"], g["draw"], 1, y_obs=g["y_obs"])
    np.testing.assert_array_equal(out["summ"].cpu().numpy()[:, 0], np.float32(g["y_obs"]))
    ev = P.pps_tb_events(spec, P.make_sampling(1, g["draw"], g["seed"]))
    assert int(ev["events"][0]) == g["events"] and int(ev["status"][0]) == 0


def test_tb_abc_top_fraction(P, torch):
    spec = W.tb_spec(n_stop=600, n_sample=100)
    y = oracle.tb_simulate(W.tb_point_spec(n_stop=600, n_sample=100), 0, 2, 1)["summ"][0]
    n = 2000
    r = P.abc(spec, y, W.SAMPLING_SEED, 0, n, P.PPS_EPS_TOP_FRACTION, 0.02)
    ref = oracle.abc(spec, y, W.SAMPLING_SEED, 0, n, oracle.EPS_TOP_FRACTION, 0.02)
    assert r["n_accepted"] == ref["n_accepted"] == 40
    sim = oracle.simulate(spec, W.SAMPLING_SEED, 0, n, y_obs=y)
    eps = ref["eps_used"]
    band = set(np.nonzero(np.abs(sim["dist"] - eps) <= 4 * DIST_TOL * max(eps, 1e-3))[0].tolist())
    got = set(r["idx"].cpu().numpy().astype(np.int64).tolist())
    assert got ^ set(ref["idx"].astype(np.int64).tolist()) <= band
    if got == set(ref["idx"].astype(np.int64).tolist()):
        np.testing.assert_allclose(r["mean"][:3], ref["mean"], rtol=1e-12)
        np.testing.assert_array_equal(r["theta"].cpu().numpy().T, ref["theta"].astype(np.float32))


def test_tb_tally_and_pvalue(P, torch):
    spec = W.tb_spec(n_stop=500, n_sample=80)
    n = 1200
    obs = np.array([0.3, 0.9])
    counts = P.pps_summary_tally(spec, P.make_sampling(n, 0, 4), obs)
    ref = oracle.summary_tally(spec, 4, 0, n, obs)
    np.testing.assert_array_equal(counts, ref)
    lam = [0.03, 0.06735, 0.12]
    c, p = P.prior_pred_pvalue(spec, 2, P.PPS_NORMAL, lam, P.make_sampling(n, 0, 4), 0.6)
    ro = oracle.pvalue(spec, 2, "normal", lam, 4, 0, n, 0.6)
    np.testing.assert_array_equal(np.asarray(c, np.int64), ro["count_ge"].astype(np.int64))


def test_tb_full_size_sampled(P, torch):
    """The benchmark run (K = 10000, n = 473, cap 2^20): events and status
    of all 16000 draws are computed on the device; 24 draws (seeded picks)
    against the oracle, exactly."""
    spec = W.tb_spec(n_stop=W.TB_PPS["n_stop"], n_sample=W.TB_PPS["n_sample"],
                     max_events=W.TB_PPS["max_events"])
    n = W.TB_PPS["n"]
    ev = P.pps_tb_events(spec, P.make_sampling(n, 0, W.SAMPLING_SEED))
    evn, stn = ev["events"].cpu().numpy(), ev["status"].cpu().numpy()
    rng = np.random.default_rng(3)
    for start in rng.choice(n - 8, size=3, replace=False):
        o = oracle.tb_simulate(spec, W.SAMPLING_SEED, int(start), 8)
        np.testing.assert_array_equal(stn[start:start + 8], o["status"])
        np.testing.assert_array_equal(evn[start:start + 8].astype(np.uint64), o["events"])
    print("full batch: complete/extinct/truncated", np.bincount(stn, minlength=3).tolist(),
          "events", int(evn.sum()))


def test_tb_invalid(P, torch):
    with pytest.raises(P.PPSError):
        P.simulate(W.tb_spec(n_stop=P.PPS_TB_MAX_POP + 1), 1, 0, 4)
