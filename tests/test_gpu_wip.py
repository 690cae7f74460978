"""Parity of the weak-informativity test (Sec. 4.1: Alg. 2 with the adaptive
SMC evidence of Alg. 3, one FP64 sampler per workgroup) with the FP64 oracle,
through the C ABI.

Bar: both sides compute in FP64 on the same random numbers and take the same
discrete decisions (tempering bisection, resampling ancestors on integer
weights, Metropolis-Hastings accepts) unless a compared quantity lies within
rounding (~1e-15 relative) of its threshold.  So a run's log evidence agrees to
WIP_TOL relative unless such a tie flipped one decision, which changes the
estimate by a Monte Carlo amount; at most a small fraction of runs may do so
(WIP_FLIP_FRAC), each still within WIP_MC of the oracle.  p-values and cut-offs
are equal where the log evidences agree.
"""
import numpy as np
import pytest

import oracle
import pps_workloads as W
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

WIP_TOL = 1e-9
WIP_FLIP_FRAC = 0.02
WIP_MC = 2.0
SPEC = W.BIOASSAY


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    return P


def compare(gpu, ref, label):
    d = np.abs(gpu - ref)
    bad = d > WIP_TOL * np.maximum(1.0, np.abs(ref))
    print(f"{label}: {len(d)} runs, max |diff| among agreeing {d[~bad].max() if (~bad).any() else 0:.2e}, "
          f"{bad.sum()} differ (max {d.max():.2e})")
    assert bad.mean() <= WIP_FLIP_FRAC
    assert np.all(d[bad] < WIP_MC)


def sets_and_lambdas(n, seed):
    lam = W.wip_lambdas(n, seed=seed)[1:]
    ys = np.array([oracle.bio_simulate(SPEC, lam[s], seed, s, oracle.P_DATA_K)[0] for s in range(n)])
    return ys, lam


@pytest.mark.parametrize("n_particles", [500, 100, 1000, 2])
def test_smc_evidence(P, torch, n_particles):
    n = 48 if n_particles <= 500 else 16
    ys, lam = sets_and_lambdas(n, 21)
    cfg = dict(W.SMC_CONFIG)
    cfg["n_particles"] = n_particles
    g = P.pps_smc_log_evidence(SPEC, ys, lam, cfg, 5, first_run=1000).cpu().numpy()
    ref = np.array([oracle.smc_log_evidence(SPEC, ys[s], lam[s], cfg, 5, 1000 + s)["log_z"]
                    for s in range(n)])
    assert np.all(np.isfinite(g))
    compare(g, ref, f"N_p={n_particles}")


def test_wip_small(P, torch):
    lam = W.wip_lambdas(3, seed=4)
    cfg = dict(W.SMC_CONFIG)
    cfg["n_particles"] = 200
    n = 40
    g = P.pps_wip_test(SPEC, lam, n, cfg, 8, 0.1)
    ref = oracle.wip_test(SPEC, lam, n, cfg, 8, 0.1)
    z0, zk = g["log_z0"].cpu().numpy(), g["log_zk"].cpu().numpy()
    compare(np.concatenate([z0.ravel(), zk.ravel()]),
            np.concatenate([ref["log_z0"].ravel(), ref["log_zk"].ravel()]), "weak-informativity K=3 N=40")
    # where every evidence agrees, the p-values and cut-offs are the oracle's
    close = (np.abs(z0 - ref["log_z0"]) <= WIP_TOL * np.abs(ref["log_z0"])).all(axis=1) & \
            (np.abs(zk - ref["log_zk"]) <= WIP_TOL * np.abs(ref["log_zk"])).all(axis=1)
    assert close.sum() >= lam.shape[0] - 1
    pv = g["pvalues"].cpu().numpy()
    for k in np.nonzero(close)[0]:
        np.testing.assert_array_equal(pv[k], ref["pvalues"][k])
        assert g["gamma"][k] == ref["gamma"][k]
    # the cut-offs are the alpha quantiles of the device p-values in every row
    for k in range(lam.shape[0]):
        assert g["gamma"][k] == np.quantile(pv[k], 0.1, method="inverted_cdf")


def test_wip_full_size_sampled(P, torch):
    """K = 400 hyperparameters, N = 400 data sets, N_p = 500 (the paper's run):
    24 sampled evidences against the oracle's single runs."""
    lam = W.wip_lambdas(W.WIP_TEST["n_lambda"], seed=W.WIP_TEST["seed"])
    n = W.WIP_TEST["n_data"]
    seed = W.WIP_TEST["seed"]
    cfg = W.SMC_CONFIG
    g = P.pps_wip_test(SPEC, lam, n, cfg, seed, W.WIP_ALPHA, with_pvalues=False)
    z0, zk = g["log_z0"].cpu().numpy(), g["log_zk"].cpu().numpy()
    assert np.all(np.isfinite(z0)) and np.all(np.isfinite(zk))
    rng = np.random.default_rng(0)
    got, ref = [], []
    for _ in range(24):
        k, i, kind = int(rng.integers(0, lam.shape[0])), int(rng.integers(0, n)), int(rng.integers(0, 2))
        if kind == 0:
            y, _ = oracle.bio_simulate(SPEC, lam[0], seed, i, oracle.P_DATA_BASE)
        else:
            y, _ = oracle.bio_simulate(SPEC, lam[k], seed, k * n + i, oracle.P_DATA_K)
        r = oracle.smc_log_evidence(SPEC, y, lam[k], cfg, seed, (k * n + i) * 2 + kind)
        got.append((z0 if kind == 0 else zk)[k, i])
        ref.append(r["log_z"])
    compare(np.array(got), np.array(ref), "full size, sampled")
    # cut-offs: the alpha quantile of each row's p-values from the device evidences
    q = int(np.ceil(W.WIP_ALPHA * n))
    for k in range(0, lam.shape[0], 50):
        p = np.searchsorted(np.sort(zk[k]), z0[k], side="right") / n
        assert g["gamma"][k] == np.sort(p)[q - 1]


def test_wip_invalid(P, torch):
    cfg = dict(W.SMC_CONFIG)
    cfg["n_particles"] = 2000
    with pytest.raises(P.PPSError):
        P.pps_wip_test(SPEC, W.wip_lambdas(2), 10, cfg, 1, 0.05)
