"""Pins of the oracle's genetic toggle switch (Sec. 3.2, Eqs. gene_uv_SDE,
gene_uv_SDE_EM, gene_u_obs) against facts fixed outside its code:

* with beta = 0 the Hill terms are constants and the Euler-Maruyama recursion
  is linear, so the final level has the closed form of a linear recursion
  driven by the cell's normals (variation of constants);
* with one gene linear, the other gene's recursion is linear in its own level
  with a known input, the Hill function of the first gene's level *before* each
  step -- again a closed form;
* the measurement model's dependence on mu, sigma and gamma (ratios that hold
  for any level u), and the index of its normal;
* the boundary at 1 (levels and measurements);
* the 19 summaries equal numpy's inverse-ECDF quantiles of the cell values;
* the 7 uniform priors' moments.
"""
import math

import numpy as np
import pytest

import oracle
import pps_workloads as W

SEED, DRAW = 7, 3


def cell_normals(cell, count, seed=SEED, draw=DRAW):
    return np.array([oracle.cell_normal(seed, draw, cell, n) for n in range(count)])


def linear_level(x0, a, drive):
    """Closed form of x_{j+1} = a x_j + drive_j: every x_j, j = 0..S."""
    s = len(drive)
    powers = a ** np.arange(s, -1, -1, dtype=np.float64)  # a^S .. a^0
    out = np.empty(s + 1)
    out[0] = x0
    # x_j = a^j x0 + sum_{l<j} a^{j-1-l} drive_l, evaluated as a direct sum
    for j in range(1, s + 1):
        out[j] = a ** j * x0 + np.dot(powers[s - j + 1:], drive[:j])
    return out


def spec_at(theta, **kw):
    return W.toggle_point_spec(theta=theta, **kw)


@pytest.mark.parametrize("dt,steps", [(1.0, 120), (0.5, 200)])
def test_linear_case_closed_form(dt, steps):
    alpha_u, alpha_v, mu = 50.0, 40.0, 300.0
    theta = (mu, 0.0, 0.1, alpha_u, alpha_v, 0.0, 0.0)
    sp = spec_at(theta, n_cells=5, steps=steps, dt=dt)
    cells = oracle.toggle_cells(sp, theta, SEED, DRAW)
    a = 1.0 - 0.03 * dt
    for c in range(5):
        z = cell_normals(c, 2 * steps)
        for level, alpha, xi in (("u", alpha_u, z[0::2]), ("v", alpha_v, z[1::2])):
            drive = dt * (alpha / 2.0 - 1.0) + 0.5 * math.sqrt(dt) * xi
            path = linear_level(10.0, a, drive)
            assert path.min() > 1.5  # the boundary never acts
            np.testing.assert_allclose(cells[level][c], path[-1], rtol=1e-12)
        # sigma = 0: the measurement is the level shifted by mu
        np.testing.assert_allclose(cells["y"][c], cells["u"][c] + mu, rtol=1e-14)


@pytest.mark.parametrize("driven", ["u", "v"])
def test_hill_term_uses_levels_before_the_step(driven):
    """One gene linear (beta = 0), the other driven through alpha / (1 +
    level^beta) by the linear gene's level before each step."""
    dt, steps, beta = 0.5, 150, 0.7
    if driven == "u":
        theta = (300.0, 0.0, 0.1, 50.0, 3.2, beta, 0.0)
    else:
        theta = (300.0, 0.0, 0.1, 3.2, 50.0, 0.0, beta)
    sp = spec_at(theta, n_cells=3, steps=steps, dt=dt)
    cells = oracle.toggle_cells(sp, theta, SEED, DRAW)
    a = 1.0 - 0.03 * dt
    for c in range(3):
        z = cell_normals(c, 2 * steps)
        xi_u, xi_v = z[0::2], z[1::2]
        lin_xi, drv_xi = (xi_v, xi_u) if driven == "u" else (xi_u, xi_v)
        lin = linear_level(10.0, a, dt * (3.2 / 2.0 - 1.0) + 0.5 * math.sqrt(dt) * lin_xi)
        hill = 50.0 / (1.0 + np.power(lin[:-1], beta))
        drv = linear_level(10.0, a, dt * hill - dt + 0.5 * math.sqrt(dt) * drv_xi)
        assert lin.min() > 1.5 and drv.min() > 1.5
        other = "v" if driven == "u" else "u"
        np.testing.assert_allclose(cells[other][c], lin[-1], rtol=1e-12)
        np.testing.assert_allclose(cells[driven][c], drv[-1], rtol=1e-12)


def test_measurement_model_ratios():
    """y = u + mu (1 + sigma eta u^-gamma): the levels do not depend on (mu,
    sigma, gamma); y - u scales with mu; the noise part scales with sigma and
    with u^-gamma; and eta is normal 2S of the cell's stream."""
    base = (300.0, 0.2, 0.1, 30.0, 20.0, 2.5, 3.5)
    steps, n_cells = 100, 200
    res = {}
    for name, th in {"base": base, "mu2": (600.0,) + base[1:],
                     "sig2": (300.0, 0.4) + base[2:], "gam2": (300.0, 0.2, 0.3) + base[3:],
                     "gam0": (300.0, 0.2, 0.0) + base[3:]}.items():
        res[name] = oracle.toggle_cells(spec_at(th, n_cells=n_cells, steps=steps), th, SEED, DRAW)
    u = res["base"]["u"]
    for r in res.values():
        np.testing.assert_array_equal(r["u"], u)
        np.testing.assert_array_equal(r["v"], res["base"]["v"])
    ok = res["base"]["y"] > 1.0
    ok &= res["mu2"]["y"] > 1.0
    ok &= res["sig2"]["y"] > 1.0
    ok &= res["gam2"]["y"] > 1.0
    assert ok.sum() > 0.9 * n_cells
    d = res["base"]["y"] - u
    np.testing.assert_allclose((res["mu2"]["y"] - u)[ok], 2.0 * d[ok], rtol=1e-12)
    noise = d - 300.0
    np.testing.assert_allclose((res["sig2"]["y"] - u - 300.0)[ok], 2.0 * noise[ok], rtol=1e-9)
    np.testing.assert_allclose((res["gam2"]["y"] - u - 300.0)[ok],
                               noise[ok] * u[ok] ** -0.2, rtol=1e-9)
    eta = (res["gam0"]["y"] - u - 300.0) / (300.0 * 0.2)
    idx = np.nonzero(res["gam0"]["y"] > 1.0)[0][:20]
    for c in idx:
        np.testing.assert_allclose(eta[c], oracle.cell_normal(SEED, DRAW, int(c), 2 * steps),
                                   rtol=1e-9, atol=1e-12)


def test_boundary_at_one():
    """alpha = 0: both genes decay onto the boundary 1 and stay at or above
    it; measurements below 1 are held at 1 (eta < -(1 + 1/mu)/sigma at u = 1)."""
    mu, sigma = 250.0, 0.5
    theta = (mu, sigma, 0.35, 0.0, 0.0, 3.0, 3.0)
    n_cells = 4000
    cells = oracle.toggle_cells(spec_at(theta, n_cells=n_cells, steps=300), theta, SEED, DRAW)
    assert cells["u"].min() == 1.0 and cells["v"].min() == 1.0
    assert (cells["u"] == 1.0).mean() > 0.3
    assert cells["y"].min() == 1.0
    at_one = cells["u"] == 1.0
    p = 0.5 * math.erfc((1.0 + 1.0 / mu) / sigma / math.sqrt(2.0))
    n1 = int(at_one.sum())
    k = int((cells["y"][at_one] == 1.0).sum())
    assert abs(k - n1 * p) < 5.0 * math.sqrt(n1 * p * (1 - p)) + 1


@pytest.mark.parametrize("n_cells", [8000, 999, 7])
def test_quantile_summaries_are_inverse_ecdf(n_cells):
    sp = W.toggle_spec(n_cells=n_cells, steps=60)
    r = oracle.simulate(sp, SEED, DRAW, 1)
    y = oracle.toggle_cells(sp, r["theta"][0], SEED, DRAW)["y"]
    levels = np.arange(1, 20) / 20.0
    ref = np.quantile(y, levels, method="inverted_cdf")
    np.testing.assert_array_equal(r["summ"][0], ref)


def test_seven_uniform_priors():
    sp = W.toggle_spec(n_cells=1, steps=1)
    th = np.array([oracle.prior_draw(sp, SEED, i)[0] for i in range(20000)])
    for j, (_, lo, hi) in enumerate(W.TOGGLE_PRIORS):
        assert th[:, j].min() >= lo and th[:, j].max() <= hi
        m, v = (lo + hi) / 2.0, (hi - lo) ** 2 / 12.0
        assert abs(th[:, j].mean() - m) < 5.0 * math.sqrt(v / len(th))
        assert abs(th[:, j].var() / v - 1.0) < 0.05
    # the parameters are independent (different prior blocks)
    c = np.corrcoef(th.T)
    assert np.abs(c - np.eye(7)).max() < 0.05


def test_cell_streams_are_distinct():
    z = np.array([[oracle.cell_normal(SEED, DRAW, c, n) for n in range(8)] for c in range(4)])
    assert len(np.unique(z)) == z.size
    assert oracle.cell_normal(SEED, DRAW, 0, 0) != oracle.path_normal(SEED, DRAW, 0)
