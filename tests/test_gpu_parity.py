"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (from the method's definition and the precision split: FP32 simulation,
FP64 priors / tallies / moments):
  * random streams: bit-exact;
  * prior draws: the FP32 theta equals the oracle's FP64 theta rounded to
    FP32 (uniform priors are computed with the same IEEE operations);
  * summaries, distance, statistic: within 1e-5 relative of the oracle;
  * accept sets: identical except draws whose oracle distance lies within
    1e-5 * eps of eps;
  * p-value tallies: identical counts over draws whose EM map is contracting
    (th1 dt < 2); decisions of chaotic draws are counted and reported.
"""
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
    return P


def test_philox_bit_exact(P, torch):
    for seed, first, block, purpose, n in [(1, 0, 0, 0, 3000), (0xDEADBEEFCAFEF00D, 2**32 - 1000, 249, 1, 2500),
                                            (7, 123456789, 3, 0, 1001)]:
        out = torch.empty(4 * n, dtype=torch.int32, device="cuda")
        P.pps_philox(seed, first, n, block, purpose, out)
        got = out.cpu().numpy().view(np.uint32).reshape(n, 4)
        ref = np.array([oracle.stream_block(seed, first + q, block, purpose) for q in range(n)])
        np.testing.assert_array_equal(got, ref)


def test_philox_known_answers(P, torch):
    from test_oracle_rng import PHILOX_KAT
    for ctr, key, expect in PHILOX_KAT:
        out = torch.empty(4, dtype=torch.int32, device="cuda")
        P.pps_philox(key[0] | (key[1] << 32), ctr[2] | (ctr[3] << 32), 1, ctr[0], ctr[1], out)
        assert out.cpu().numpy().view(np.uint32).tolist() == list(expect)


@pytest.mark.parametrize("m", [22, 25, 29])  # 4, 1 and 5 normals past whole blocks of six
def test_path_normals_fp32_vs_fp64(P, torch, m):
    seed, first, n = 3, 2**32 - 37, 1500  # draw indices cross the 2^32 boundary
    out = torch.empty((m, n), dtype=torch.float32, device="cuda")
    P.pps_normals(seed, first, n, m, out)
    got = out.cpu().numpy().astype(np.float64)
    ref = np.array([[oracle.path_normal(seed, first + q, k) for q in range(n)] for k in range(m)])
    err = np.abs(got - ref)
    print("normals: max abs err", err.max(), "max rel err", (err / np.maximum(np.abs(ref), 1)).max())
    assert err.max() < 2e-5 * max(1.0, np.abs(ref).max())


def _logistic_parity(P, spec, seed, first, n, y):
    g = P.simulate(spec, seed, first, n, y_obs=y)
    o = oracle.simulate(spec, seed, first, n, y_obs=y)
    th = g["theta"].cpu().numpy().T
    np.testing.assert_array_equal(th, o["theta"].astype(np.float32))
    summ = g["summ"].cpu().numpy().T
    scale = np.abs(o["summ"]).max()
    e_obs = rel_err(summ, o["summ"], floor=1e-3 * scale)
    e_d = rel_err(g["dist"].cpu().numpy(), o["dist"])
    e_t = rel_err(g["stat"].cpu().numpy(), o["stat"], floor=1e-3 * scale)
    print(f"logistic S={spec['steps']} n={n}: obs {e_obs.max():.2e} dist {e_d.max():.2e} "
          f"stat {e_t.max():.2e}")
    assert e_obs.max() <= TOL and e_d.max() <= TOL and e_t.max() <= TOL
    return g, o


def test_logistic_summaries_ragged(P, torch):
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=1000)
    _logistic_parity(P, spec, W.SAMPLING_SEED, 0, 5003, y)  # 19.5 tiles of 256


# step counts with every remainder modulo 6 (the normals of a Philox block)
@pytest.mark.parametrize("steps,n_obs,t_end", [(20, 4, 2.0), (200, 20, 10.0), (5000, 20, 10.0), (30, 3, 1.0),
                                               (25, 5, 2.0), (35, 7, 2.0), (9, 3, 1.0)])
def test_logistic_step_counts(P, torch, steps, n_obs, t_end):
    spec = W.logistic_spec(steps=steps, n_obs=n_obs, t_end=t_end)
    y = np.linspace(20, 90, n_obs)
    n = 700 if steps >= 5000 else 1337
    _logistic_parity(P, spec, 9, 77, n, y)


def test_self_distance_point_priors(P, torch):
    ob = observed()["logistic_S1000"]
    spec = W.logistic_point_spec(steps=1000)
    g = P.simulate(spec, 0, 0, 1, y_obs=ob["y_obs"])
    d = float(g["dist"][0])
    print("self distance", d, "norm", np.linalg.norm(ob["y_obs"]))
    assert d <= 1e-5 * np.linalg.norm(ob["y_obs"])


@pytest.mark.parametrize("m", [20, 1, 6, 7, 11])
def test_normal_mean_summaries(P, torch, m):
    spec = W.normal_mean_spec(n_obs=m, noise_sd=1.5, prior_sd=2.0)
    g = P.simulate(spec, 5, 11, 3001, y_obs=np.zeros(m))
    o = oracle.simulate(spec, 5, 11, 3001, y_obs=np.zeros(m))
    np.testing.assert_array_equal(g["theta"].cpu().numpy().T, o["theta"].astype(np.float32))
    err = np.abs(g["summ"].cpu().numpy().T - o["summ"])
    assert err.max() <= 1e-5 * np.abs(o["summ"]).max()


def test_abc_top_fraction_small_workload(P, torch):
    """N = 1e4, closest 1%: accept set, eps and FP64 posterior moments."""
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=1000)
    n, frac = W.ABC_SMALL["n"], W.ABC_SMALL["frac"]
    g = P.abc(spec, y, W.SAMPLING_SEED, 0, n, P.PPS_EPS_TOP_FRACTION, frac)
    o = oracle.abc(spec, y, W.SAMPLING_SEED, 0, n, oracle.EPS_TOP_FRACTION, frac)
    assert g["n_accepted"] == o["n_accepted"] == 100
    assert abs(g["eps_used"] - o["eps_used"]) <= TOL * o["eps_used"]
    gi = g["idx"].cpu().numpy()
    assert np.all(np.diff(gi) > 0)  # increasing draw index
    sim = oracle.simulate(spec, W.SAMPLING_SEED, 0, n, y_obs=y)
    eps = o["eps_used"]
    band = set(np.nonzero(np.abs(sim["dist"] - eps) <= TOL * eps)[0].tolist())
    diff = set(gi.tolist()) ^ set(o["idx"].tolist())
    assert diff <= band, (diff, band)
    if not diff:
        np.testing.assert_allclose(g["mean"][:3], o["mean"], rtol=1e-12)
        np.testing.assert_allclose(g["var"][:3], o["var"], rtol=1e-10)
        np.testing.assert_array_equal(g["theta"].cpu().numpy().T, o["theta"].astype(np.float32))
        np.testing.assert_allclose(g["dist"].cpu().numpy(), o["dist"], rtol=TOL)


def test_abc_fixed_eps_and_truncation(P, torch):
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=200)
    n = 9000
    sim = oracle.simulate(spec, 4, 1000, n, y_obs=y)
    eps = float(np.quantile(sim["dist"], 0.05))
    g = P.abc(spec, y, 4, 1000, n, P.PPS_EPS_FIXED, eps)
    ref = np.nonzero(sim["dist"] <= eps)[0] + 1000
    band = set((np.nonzero(np.abs(sim["dist"] - eps) <= TOL * eps)[0] + 1000).tolist())
    got = g["idx"].cpu().numpy()
    assert set(got.tolist()) ^ set(ref.tolist()) <= band
    assert g["eps_used"] == eps
    # truncation: first `capacity` by index, true count reported
    t = P.abc(spec, y, 4, 1000, n, P.PPS_EPS_FIXED, eps, capacity=7)
    assert t["status"] == P.PPS_ETRUNC and t["n_accepted"] == g["n_accepted"]
    np.testing.assert_array_equal(t["idx"].cpu().numpy(), got[:7])
    np.testing.assert_allclose(t["mean"], g["mean"], rtol=0, atol=0)
    # capacity 0: statistics only
    z = P.abc(spec, y, 4, 1000, n, P.PPS_EPS_FIXED, eps, capacity=0)
    assert z["n_accepted"] == g["n_accepted"]


def test_abc_ties_by_index(P, torch):
    spec = W.logistic_spec(steps=100, theta1=("point", 1, 0), theta2=("point", 100, 0),
                           theta3=("point", 0.0, 0))
    g = P.abc(spec, np.full(20, 50.0), 1, 10, 3000, P.PPS_EPS_TOP_FRACTION, 0.05)
    np.testing.assert_array_equal(g["idx"].cpu().numpy(), np.arange(10, 160))
    assert g["n_accepted"] == 150


def test_abc_single_draw_and_full_fraction(P, torch):
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=100)
    g = P.abc(spec, y, 2, 5, 1, P.PPS_EPS_TOP_FRACTION, 0.01)
    assert g["n_accepted"] == 1 and int(g["idx"][0]) == 5 and math.isnan(g["var"][0])
    g = P.abc(spec, y, 2, 0, 777, P.PPS_EPS_TOP_FRACTION, 1.0)
    assert g["n_accepted"] == 777
    np.testing.assert_array_equal(g["idx"].cpu().numpy(), np.arange(777))


def _chaotic(theta1, dt):
    return theta1 * dt >= 2.0


def test_pvalue_lambda_grid_parity(P, torch):
    """64-lambda grid at reduced N: counts equal up to chaotic-draw flips."""
    spec = W.pvalue_spec(steps=1000)
    t_obs = observed()["logistic_S1000"]["t_obs"]
    lam = W.lambda_grid(64)
    n = 3000
    counts, p = P.prior_pred_pvalue(spec, 0, P.PPS_LOGNORMAL, lam, P.make_sampling(n, 0, 1), t_obs)
    ref = oracle.pvalue(spec, 0, "lognormal", lam, 1, 0, n, t_obs)
    np.testing.assert_array_equal(p, counts / n)
    flips_total = 0
    for k in (0, 20, 40, 63):
        sk = dict(spec, priors=[("lognormal", 0.0, float(lam[k]))] + spec["priors"][1:])
        o = oracle.simulate(sk, 1, 0, n)
        g = P.simulate(sk, 1, 0, n)
        dec_o = o["stat"] >= t_obs
        dec_g = g["stat"].cpu().numpy().astype(np.float64) >= t_obs
        chaotic = _chaotic(o["theta"][:, 0], 0.01)
        assert np.array_equal(dec_o[~chaotic], dec_g[~chaotic]), k
        flips_total += int((dec_o != dec_g).sum())
        assert int(dec_g.sum()) == int(counts[k])
    diff = np.abs(counts.astype(np.int64) - ref["count_ge"].astype(np.int64))
    print("p-value count differences per lambda:", diff.max(), "flips in sampled lambdas:", flips_total)
    small = lam <= 1.0
    np.testing.assert_array_equal(counts[small], ref["count_ge"][small])
    assert diff.max() <= max(3, int(2e-3 * n))


# step counts 4, 0 and 2 modulo 6 (the normals of a Philox block)
@pytest.mark.parametrize("lp,family,lams,steps", [
    (0, "lognormal", list(W.lambda_grid(37)), 400),                 # one group + 5 rows
    (1, "uniform", [60.0 + 1.5 * k for k in range(33)], 420),       # th2 ~ U(50, lambda)
    (2, "uniform", [0.05 + 0.006 * k for k in range(70)], 440),     # th3 ~ U(0, lambda), 2 groups + 6
])
def test_pvalue_lambda_groups_equal_single_rows(P, torch, lp, family, lams, steps):
    """Grids run in groups of 32 lambda values per lane (shared random numbers);
    every count equals the one-lambda-per-row result, remainder rows included."""
    spec = W.pvalue_spec(steps=steps)
    fam = {"lognormal": P.PPS_LOGNORMAL, "uniform": P.PPS_UNIFORM}[family]
    t_obs = observed()["logistic_S1000"]["t_obs"]
    s = P.make_sampling(5003, 17, 4)
    counts, _ = P.prior_pred_pvalue(spec, lp, fam, lams, s, t_obs)
    single = [int(P.prior_pred_pvalue(spec, lp, fam, [l], s, t_obs)[0][0]) for l in lams]
    np.testing.assert_array_equal(counts.astype(np.int64), np.array(single))
    ref = oracle.pvalue(spec, lp, family, lams, 4, 17, 5003, t_obs)
    assert np.abs(counts.astype(np.int64) - ref["count_ge"].astype(np.int64)).max() <= 3


def test_conjugate_normal_pvalue_gpu(P, torch):
    spec = W.normal_mean_spec(n_obs=20, noise_sd=1.0)
    n, t_obs = 200000, 0.4
    lam = [0.3, 1.0, 2.0]
    counts, p = P.prior_pred_pvalue(spec, 0, P.PPS_NORMAL, lam, P.make_sampling(n, 0, 21), t_obs)
    ref = oracle.pvalue(spec, 0, "normal", lam, 21, 0, n, t_obs)
    np.testing.assert_array_equal(counts, ref["count_ge"])
    for k, l in enumerate(lam):
        pe = 1 - 0.5 * math.erfc(-(t_obs / math.sqrt(l * l + 1 / 20)) / math.sqrt(2))
        assert abs(p[k] - pe) <= 4 * math.sqrt(pe * (1 - pe) / n)


GARCH_TOL = 1e-5
GARCH_NAMES = ("mean", "var", "skew", "kurt", "acf")


def garch_scales(spec, seed, draws):
    """Per draw and summary, the magnitude the 1e-5 bar is relative to: the
    value for variance and kurtosis, the sum over absolute terms for the
    signed mean and skewness, 1 for the ACFs."""
    return oracle.garch_bar_scales(spec, seed, draws)


def garch_errors(g, o, scale):
    """Per-summary errors in units of the scale above (the bar is 1e-5)."""
    e = np.abs(g - o) / scale
    return {"mean": e[:, 0], "var": e[:, 1], "skew": e[:, 2], "kurt": e[:, 3],
            "acf": e[:, 4:].max(axis=1)}


# lengths 0, 20 and 40 modulo 60 (the kernel's spans of ten Philox blocks;
# 40: no whole span).  Not 20: the ACF of a 20-step series is conditioned so
# badly that FP32 sums in the kernel's order, emulated on the CPU with the
# oracle's normals, already miss the 1e-5 bar (2.0e-5; 4.8e-6 at 40 steps).
@pytest.mark.parametrize("length", [2000, 120, 160, 40])
def test_garch_summaries(P, torch, length):
    spec = W.garch_spec(series_len=length)
    n = 2003
    g = P.simulate(spec, 1, 0, n)
    o = oracle.simulate(spec, 1, 0, n)
    np.testing.assert_array_equal(g["theta"].cpu().numpy().T, o["theta"].astype(np.float32))
    gs = g["summ"].cpu().numpy().T.astype(np.float64)
    errs = garch_errors(gs, o["summ"], garch_scales(spec, 1, range(n)))
    for k, e in errs.items():
        print(f"GARCH {k}: max {e.max():.2e} median {np.median(e):.2e} p99 {np.quantile(e, 0.99):.2e}")
    for k, e in errs.items():
        assert e.max() <= GARCH_TOL, k


def test_garch_tally(P, torch):
    """Tail-area tallies equal the oracle's except for draws whose oracle
    summary lies within the summary bar of the observed value."""
    spec = W.garch_spec()
    obs = np.array(observed()["garch_L2000"]["summaries"])
    n = 3000
    counts = P.pps_summary_tally(spec, P.make_sampling(n, 0, 1), obs)
    ref = oracle.summary_tally(spec, 1, 0, n, obs)
    summ = oracle.simulate(spec, 1, 0, n)["summ"]
    near = (np.abs(summ - obs[None, :]) <= GARCH_TOL * garch_scales(spec, 1, range(n))).sum(axis=0)
    diff = np.abs(counts.astype(np.int64) - ref.astype(np.int64))
    print("GARCH tallies", counts, ref, "near ties", near)
    assert np.all(diff <= near), (diff, near)


def test_sharding_invariance(P, torch):
    """[0, N) equals [0, N/2) + [N/2, N) bit for bit."""
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=200)
    a = P.simulate(spec, 3, 0, 4000, y_obs=y)
    b = P.simulate(spec, 3, 0, 1700, y_obs=y)
    c = P.simulate(spec, 3, 1700, 2300, y_obs=y)
    for key in ("theta", "summ"):
        np.testing.assert_array_equal(a[key].cpu().numpy(),
                                      np.concatenate([b[key].cpu().numpy(), c[key].cpu().numpy()], axis=1))
    for key in ("stat", "dist"):
        np.testing.assert_array_equal(a[key].cpu().numpy(),
                                      np.concatenate([b[key].cpu().numpy(), c[key].cpu().numpy()]))


def test_launch_shape_invariance(P, torch):
    """Every supported launch shape (workgroup size, draws per lane, Philox
    blocks per loop trip) gives bit-identical per-draw results and ABC output."""
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=200)
    n = 3001
    keep = P.pps_get_launch_shape(0)
    try:
        ref = None
        for shape in P.PATH_SHAPES:
            P.pps_set_launch_shape(0, *shape)
            g = P.simulate(spec, 8, 5, n, y_obs=y)
            a = P.abc(spec, y, 8, 5, n, P.PPS_EPS_TOP_FRACTION, 0.02)
            cur = [g[k].cpu().numpy() for k in ("theta", "summ", "stat", "dist")] + \
                  [a["idx"].cpu().numpy(), a["theta"].cpu().numpy(), a["dist"].cpu().numpy(),
                   np.array([a["eps_used"]]), a["mean"], a["var"]]
            if ref is None:
                ref = cur
            else:
                for x, r in zip(cur, ref):
                    np.testing.assert_array_equal(x, r, err_msg=str(shape))
    finally:
        P.pps_set_launch_shape(0, *keep)
    keep = P.pps_get_launch_shape(1)
    try:
        gs = W.garch_spec(series_len=200)
        ref = None
        for shape in P.GARCH_SHAPES:
            P.pps_set_launch_shape(1, *shape)
            cur = P.simulate(gs, 2, 0, 1500)["summ"].cpu().numpy()
            if ref is None:
                ref = cur
            else:
                np.testing.assert_array_equal(cur, ref, err_msg=str(shape))
    finally:
        P.pps_set_launch_shape(1, *keep)


def test_autotune_and_cache(P, torch, tmp_path, monkeypatch):
    """The autotuner times every supported shape, applies the fastest, and a
    cache hit applies the recorded shape without timing."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PPS_TUNE_CACHE", str(cache))
    keep = P.pps_get_launch_shape(0)
    try:
        spec = W.logistic_spec(steps=200)
        rep = P.pps_autotune(spec, 1 << 18, use_cache=True)
        assert not rep["from_cache"] and len(rep["entries"]) == len(P.PATH_SHAPES)
        assert all(e[3] > 0 for e in rep["entries"])
        assert rep["best"] in [tuple(s) for s in P.PATH_SHAPES]
        assert P.pps_get_launch_shape(0) == rep["best"]
        line = cache.read_text().split()
        # class 0, steps bucket 256, draws bucket 2^18
        assert line[1] == "0" and line[2] == "256" and line[3] == str(1 << 18)
        P.pps_set_launch_shape(0, 64, 2, 2)
        rep2 = P.pps_autotune(spec, (1 << 17) + 1, use_cache=True)  # same buckets
        assert rep2["from_cache"] and rep2["best"] == rep["best"]
        assert P.pps_get_launch_shape(0) == rep["best"]
        # another draw count is another entry; lines of another form are skipped
        assert not P.pps_autotune(spec, 1 << 16, use_cache=True)["from_cache"]
        old = tmp_path / "old.txt"
        old.write_text(" ".join(line[:3] + line[4:]) + "\n")
        monkeypatch.setenv("PPS_TUNE_CACHE", str(old))
        assert not P.pps_autotune(spec, 1 << 18, use_cache=True)["from_cache"]
        g = P.pps_autotune(W.garch_spec(series_len=200), 1 << 15, use_cache=False)
        assert len(g["entries"]) == len(P.GARCH_SHAPES)
    finally:
        P.pps_set_launch_shape(0, *keep)


def test_invalid_arguments_raise(P, torch):
    spec = W.logistic_spec(steps=999)
    with pytest.raises(P.PPSError):
        P.simulate(spec, 1, 0, 10)
    with pytest.raises(P.PPSError):
        P.abc(W.logistic_spec(), np.zeros(20), 1, 0, 100, P.PPS_EPS_TOP_FRACTION, 1.5)


def test_kernel_timing_events(P, torch):
    """The simulation kernels are timed by HIP event-record nodes of the
    epoch's graph: with timing on, each call reports a positive kernel time
    below the call's wall time, growing with the work."""
    import time
    ob = observed()["logistic_S1000"]
    spec = W.logistic_spec(steps=1000)
    P.pps_set_timing(True)
    try:
        kms = []
        for n in (2_000_000, 8_000_000):  # both above one pass of the resident grid
            P.abc(spec, ob["y_obs"], 1, 0, n, P.PPS_EPS_FIXED, 60.0)  # first use builds the graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.abc(spec, ob["y_obs"], 1, 0, n, P.PPS_EPS_FIXED, 60.0)
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t0) * 1e3
            k = P.pps_last_kernel_ms()
            f = P.pps_last_finalize_ms()
            assert 0.0 < k <= wall_ms, (n, k, wall_ms)
            # the finalisation follows the simulation inside the same call
            assert 0.0 < f and k + f <= wall_ms, (n, k, f, wall_ms)
            kms.append(k)
        assert 2.5 * kms[0] < kms[1] < 6.0 * kms[0]
    finally:
        P.pps_set_timing(False)
