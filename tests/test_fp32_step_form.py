"""Why the FP32 Euler-Maruyama step is written in increment form (reading of
Eq. gene_uv_SDE_EM for the single-precision device path).

The logistic step X <- X + X (a - b X + c z) and its multiplicative rewrite
X <- X (1 + a - b X + c z) are equal in exact arithmetic, but in FP32 the
second rounds 1 + a (a = theta1 dt ~ 1e-2) and loses the low bits of the
drift every step.  On the same normals (rounded to FP32 for both), over the
logistic workload's priors, the increment form stays within the 1e-5
relative summary tolerance of the FP64 path at S = 1000 and 5000 steps and the
multiplicative one does not.  (numpy FP32 arithmetic, no fused operations:
the device's FMAs round less, so this is the conservative side.)
"""
import numpy as np
import pytest

import pps_workloads as W

TOL = 1e-5


def step_form_errors(steps, n=2000, seed=0):
    spec = W.logistic_spec(steps=steps, n_obs=20)
    rng = np.random.default_rng(seed)
    (_, a1, b1), (_, a2, b2), (_, a3, b3) = spec["priors"]
    th = np.stack([rng.uniform(a1, b1, n), rng.uniform(a2, b2, n), rng.uniform(a3, b3, n)], 1)
    dt = spec["t_end"] / steps
    z32 = rng.standard_normal((steps, n)).astype(np.float32)
    a64, b64, c64 = th[:, 0] * dt, th[:, 0] * dt / th[:, 1], th[:, 2] * np.sqrt(dt)
    a32, b32, c32 = (v.astype(np.float32) for v in (a64, b64, c64))
    x64 = np.full(n, spec["x0"])
    xi = np.full(n, spec["x0"], np.float32)
    xm = xi.copy()
    stride = steps // spec["n_obs"]
    ref, inc, mul = [], [], []
    for k in range(steps):
        z = z32[k]
        x64 = np.maximum(0.0, x64 + x64 * (a64 - b64 * x64 + c64 * z.astype(np.float64)))
        xi = np.maximum(np.float32(0), xi + xi * (a32 - b32 * xi + c32 * z))
        xm = np.maximum(np.float32(0), xm * (np.float32(1) + a32 - b32 * xm + c32 * z))
        if (k + 1) % stride == 0:
            ref.append(x64.copy())
            inc.append(xi.astype(np.float64))
            mul.append(xm.astype(np.float64))
    ref, inc, mul = map(np.array, (ref, inc, mul))
    ok = ref > 1e-3
    return (np.abs(inc - ref)[ok] / ref[ok]).max(), (np.abs(mul - ref)[ok] / ref[ok]).max()


@pytest.mark.parametrize("steps", [1000, 5000])
def test_increment_form_meets_the_tolerance_and_the_product_form_does_not(steps):
    e_inc, e_mul = step_form_errors(steps)
    assert e_inc < TOL / 2, e_inc
    assert e_mul > TOL, e_mul
    assert e_mul > 10 * e_inc
