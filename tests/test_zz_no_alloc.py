"""abc_sample_noalloc (through the C ABI): the allocation-free variant of
abc_sample, its scratch in the library's static device array, gives
abc_sample's records, tolerance and moments bit for bit, on two calls in a
row (the second smaller, over the first call's leftover scratch), in both
tolerance modes; sizes beyond its maximum are refused before any launch."""
import numpy as np
import pytest

import pps_workloads as W
from gpu_helpers import observed, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def P(torch):
    import paper_1902_09046_amd as P
    return P


def _noalloc(P, torch, spec, y, s, mode, arg, capacity):
    model = P.make_model(spec)
    idx = torch.full((capacity,), -1, dtype=torch.int64, device="cuda")
    th = torch.full((model.n_params, capacity), float("nan"), dtype=torch.float32, device="cuda")
    d = torch.full((capacity,), float("nan"), dtype=torch.float32, device="cuda")
    rc, st = P.abc_sample_noalloc(model, y, s, mode, arg, capacity, idx, th, d)
    k = min(st["n_accepted"], capacity)
    st.update({"status": rc, "idx": idx[:k], "theta": th[:, :k], "dist": d[:k]})
    return st


def _same(P, a, ref):
    assert a["status"] == ref["status"]
    assert a["n_accepted"] == ref["n_accepted"]
    assert a["eps_used"] == ref["eps_used"]
    np.testing.assert_array_equal(a["mean"][:3], ref["mean"][:3])
    np.testing.assert_array_equal(a["var"][:3], ref["var"][:3])
    for key in ("idx", "theta", "dist"):
        np.testing.assert_array_equal(a[key].cpu().numpy(), ref[key].cpu().numpy())


@pytest.mark.parametrize("mode", ["top", "fixed"])
def test_noalloc_equals_abc_sample(P, torch, mode):
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=400)
    m, arg = (P.PPS_EPS_TOP_FRACTION, 0.01) if mode == "top" else (P.PPS_EPS_FIXED, 60.0)
    for n, first, seed in ((300_000, 5, 7), (70_001, 12_345, 8)):
        cap = int(np.ceil(0.01 * n)) + 1 if mode == "top" else 20_000
        print(f"noalloc {mode}: n={n} first={first} seed={seed}", flush=True)
        ref = P.abc(spec, y, seed, first, n, m, arg, capacity=cap)
        got = _noalloc(P, torch, spec, y, P.make_sampling(n, first, seed), m, arg, cap)
        _same(P, got, ref)


def test_noalloc_refuses_beyond_maximum(P, torch):
    y = np.array(observed()["logistic_S1000"]["y_obs"])
    spec = W.logistic_spec(steps=200)
    P.abc(spec, y, 1, 0, 1000, P.PPS_EPS_TOP_FRACTION, 0.01)
    with pytest.raises(P.PPSError) as e:
        _noalloc(P, torch, spec, y, P.make_sampling(P.PPS_NOALLOC_MAX_DRAWS + 1, 0, 1),
                 P.PPS_EPS_TOP_FRACTION, 0.01, 16)
    assert e.value.status == P.PPS_EINVAL
    # the largest size it takes still equals abc_sample
    n = P.PPS_NOALLOC_MAX_DRAWS
    ref = P.abc(spec, y, 2, 0, n, P.PPS_EPS_TOP_FRACTION, 0.001)
    got = _noalloc(P, torch, spec, y, P.make_sampling(n, 0, 2), P.PPS_EPS_TOP_FRACTION, 0.001,
                   int(np.ceil(0.001 * n)) + 1)
    _same(P, got, ref)
