"""FP64 CPU oracle for prior-predictive sampling (arXiv:1902.09046).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does, and the two share no code: the C source here
(``pps_oracle.c``) is written independently of the HIP library, and this
wrapper marshals arguments with its own ctypes structures.

Each function follows one passage of the paper:

* ``philox`` / ``stream_block`` / ``uniform`` / ``box_muller`` -- the per-draw
  random streams (Sec. 2.5, independent streams; Philox4x32-10 from Salmon et
  al., SC'11) and the Box-Muller normal generator (Sec. 3.4 uses the
  Box-Muller method of MKL).
* ``simulate`` -- prior-predictive sampling, Eq. ppd and Alg. 1's first two
  steps: theta ~ pi(theta), D ~ s(D; theta), reduced to its summaries.
* ``abc`` -- ABC rejection in its fixed-N form (Alg. 1 and the paragraph after
  it): accept rho <= eps, or the closest fraction with eps chosen a posteriori.
* ``pvalue`` -- the prior-predictive p-value under each lambda of a
  hyperparameter grid (Eqs. pppv, pppvhype), using a tail-area statistic.
* ``summary_tally`` -- per-summary tail areas (the GARCH and toggle-switch
  checks).
* ``bio_simulate`` / ``bio_loglik`` / ``smc_log_evidence`` / ``wip_test`` --
  the weak-informativity test of Sec. 4.1 (Alg. 2) with the evidence of the
  logistic dose-response model (Eq. bioassay) estimated by the adaptive SMC
  sampler of Alg. 3 (``wip_oracle.c``).
* ``gamma_p`` / ``bege_cdf`` / ``bege_density`` / ``bege_loglik`` -- the
  log-likelihood of the BEGE volatility model (Sec. 4.2: Eqs. BEGE, shape,
  BEGE_LL, CDF_BEGE, BEGE_LL_approx, incompGamma; ``bege_oracle.c``).
* ``toggle_cells`` -- every cell of one draw of the genetic toggle switch
  (Sec. 3.2, Eqs. gene_uv_SDE, gene_uv_SDE_EM and gene_u_obs), for checks of
  its dynamics, measurement model and quantile summaries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Mapping, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "pps_oracle.c"), os.path.join(_HERE, "wip_oracle.c"),
         os.path.join(_HERE, "bege_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

UNIFORM, NORMAL, LOGNORMAL, POINT = 0, 1, 2, 3
LOGISTIC, GARCH11, NORMAL_MEAN, TOGGLE_SWITCH, TB = 0, 1, 2, 3, 4
TB_COMPLETE, TB_EXTINCT, TB_TRUNCATED = 0, 1, 2
TB_PURPOSE_EVENT, TB_PURPOSE_SAMPLE = 0x90000000, 0x90000001
MAX_PARAMS = 8
EPS_FIXED, EPS_TOP_FRACTION = 0, 1
GARCH_NSUMM = 14

_FAMILY = {"uniform": UNIFORM, "normal": NORMAL, "lognormal": LOGNORMAL, "point": POINT}
_MODEL = {"logistic": LOGISTIC, "garch11": GARCH11, "normal_mean": NORMAL_MEAN,
          "toggle_switch": TOGGLE_SWITCH, "tb": TB}


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, -O2, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(
        ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-Wall", *_SRCS, "-o", tmp, "-lquadmath", "-lm"],
        check=True,
    )
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Prior(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double)]


class _Model(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("n_params", ctypes.c_int32),
        ("prior", _Prior * MAX_PARAMS),
        ("constraint", ctypes.c_int32),
        ("x0", ctypes.c_double),
        ("t_end", ctypes.c_double),
        ("steps", ctypes.c_int32),
        ("n_obs", ctypes.c_int32),
        ("noise_sd", ctypes.c_double),
        ("n_cells", ctypes.c_int32),
    ]


class _Bioassay(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("n_trials", ctypes.c_int32 * 8),
                ("dose", ctypes.c_double * 8)]


class _SmcConfig(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int32), ("max_mcmc", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("bisect_iters", ctypes.c_int32),
                ("c", ctypes.c_double), ("h", ctypes.c_double)]


# stream purposes of the weak-informativity test (counter word 1)
P_DATA_BASE, P_DATA_K = 0x40000000, 0x40000001

_lib = None


def _check(rc: int, what: str = "invalid input") -> None:
    """Raises for a negative oracle status (-2: a buffer could not be allocated)."""
    if rc == -2:
        raise MemoryError("oracle: allocation failed")
    if rc < 0:
        raise ValueError("oracle: " + what)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        mp = ctypes.POINTER(_Model)
        lib.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.or_stream_block.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u32p]
        lib.or_uniform.argtypes = [ctypes.c_uint32]
        lib.or_uniform.restype = ctypes.c_double
        lib.or_angle_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
        lib.or_angle_uniform.restype = ctypes.c_double
        lib.or_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.or_path_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.or_path_normal.restype = ctypes.c_double
        lib.or_cell_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
        lib.or_cell_normal.restype = ctypes.c_double
        lib.or_toggle_cells.argtypes = [mp, f64p, ctypes.c_uint64, ctypes.c_uint64, f64p, f64p, f64p]
        lib.or_toggle_cells.restype = ctypes.c_int
        lib.or_prior_draw.argtypes = [mp, ctypes.c_uint64, ctypes.c_uint64, f64p]
        lib.or_prior_draw.restype = ctypes.c_int
        lib.or_n_summaries.argtypes = [mp]
        lib.or_n_summaries.restype = ctypes.c_int
        lib.or_simulate.argtypes = [mp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_void_p, f64p, f64p, f64p, f64p, i32p]
        lib.or_simulate.restype = ctypes.c_int
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        lib.or_tb_select.argtypes = [u32p, ctypes.c_int, ctypes.c_uint64]
        lib.or_tb_select.restype = ctypes.c_int
        lib.or_tb_lowest_empty.argtypes = [u32p, ctypes.c_int]
        lib.or_tb_lowest_empty.restype = ctypes.c_int
        lib.or_tb_thresholds.argtypes = [f64p, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64)]
        lib.or_tb_run.argtypes = [f64p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint64, u32p, ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64)]
        lib.or_tb_run.restype = ctypes.c_int
        lib.or_tb_summaries.argtypes = [u32p, u32p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.c_uint64, f64p]
        lib.or_tb_simulate.argtypes = [mp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, f64p,
                                       i32p, u64p, u64p, f64p]
        lib.or_tb_simulate.restype = ctypes.c_int
        lib.or_top_count.argtypes = [ctypes.c_double, ctypes.c_uint64]
        lib.or_top_count.restype = ctypes.c_uint64
        lib.or_abc.argtypes = [mp, f64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.c_int, ctypes.c_double, ctypes.c_uint64, u64p, f64p, f64p,
                               ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double),
                               f64p, f64p]
        lib.or_abc.restype = ctypes.c_int
        lib.or_pvalue.argtypes = [mp, ctypes.c_int, ctypes.c_int, f64p, ctypes.c_int, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, u64p, f64p]
        lib.or_pvalue.restype = ctypes.c_int
        lib.or_summary_tally.argtypes = [mp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, f64p, u64p]
        lib.or_summary_tally.restype = ctypes.c_int
        lib.or_logistic_path.argtypes = [mp, f64p, ctypes.c_uint64, ctypes.c_uint64, f64p]
        lib.or_logistic_path.restype = ctypes.c_int
        lib.or_garch_series.argtypes = [mp, f64p, ctypes.c_uint64, ctypes.c_uint64, f64p]
        lib.or_garch_series.restype = ctypes.c_int
        lib.or_garch_summaries.argtypes = [f64p, ctypes.c_int, f64p]
        lib.or_distance.argtypes = [f64p, f64p, ctypes.c_int]
        lib.or_distance.restype = ctypes.c_double
        lib.or_max_threads.restype = ctypes.c_int
        bp, cp = ctypes.POINTER(_Bioassay), ctypes.POINTER(_SmcConfig)
        lib.or_bio_simulate.argtypes = [bp, f64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                        i32p, f64p]
        lib.or_bio_loglik.argtypes = [bp, i32p, ctypes.c_double, ctypes.c_double]
        lib.or_bio_loglik.restype = ctypes.c_double
        lib.or_bio_logprior.argtypes = [f64p, ctypes.c_double, ctypes.c_double]
        lib.or_bio_logprior.restype = ctypes.c_double
        lib.or_smc_log_evidence.argtypes = [bp, i32p, f64p, cp, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
        lib.or_smc_log_evidence.restype = ctypes.c_double
        lib.or_wip_test.argtypes = [bp, f64p, ctypes.c_int, ctypes.c_uint64, cp, ctypes.c_uint64,
                                    ctypes.c_double, f64p, f64p, f64p, f64p]
        lib.or_wip_test.restype = ctypes.c_int
        lib.or_smc_temper.argtypes = [f64p, ctypes.c_int, ctypes.c_double, ctypes.c_int, cp]
        lib.or_smc_temper.restype = ctypes.c_double
        lib.or_smc_resample.argtypes = [f64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint32, i32p]
        lib.or_smc_proposal.argtypes = [f64p, f64p, ctypes.c_int, ctypes.c_double, f64p]
        lib.or_smc_moves.argtypes = [ctypes.c_int, ctypes.c_int, cp]
        lib.or_smc_moves.restype = ctypes.c_int
        lib.or_gamma_p.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.or_gamma_p.restype = ctypes.c_double
        d5 = [ctypes.c_double] * 5
        lib.or_gamma_q.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.or_gamma_q.restype = ctypes.c_double
        lib.or_bege_cdf.argtypes = d5 + [ctypes.c_int]
        lib.or_bege_cdf.restype = ctypes.c_double
        lib.or_bege_density.argtypes = d5 + [ctypes.c_int]
        lib.or_bege_density.restype = ctypes.c_double
        lib.or_bege_density_q.argtypes = d5 + [ctypes.c_int]
        lib.or_bege_density_q.restype = ctypes.c_double
        lib.or_bege_loglik.argtypes = [f64p, f64p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_double)]
        lib.or_bege_loglik.restype = ctypes.c_int
        lib.or_bege_loglik_batch.argtypes = [f64p, ctypes.c_int, f64p, ctypes.c_int, ctypes.c_int, f64p,
                                             ctypes.c_void_p]
        lib.or_bege_loglik_batch.restype = ctypes.c_int
        lib.or_bege_simulate.argtypes = [f64p, ctypes.c_int, ctypes.c_uint64, f64p]
        lib.or_bege_simulate.restype = ctypes.c_int
        _lib = lib
    return _lib


def _model(spec: Mapping) -> _Model:
    m = _Model()
    m.model = _MODEL[spec["model"]]
    priors = spec["priors"]
    m.n_params = len(priors)
    for j, (fam, a, b) in enumerate(priors):
        m.prior[j].family = _FAMILY[fam]
        m.prior[j].a = float(a)
        m.prior[j].b = float(b)
    m.constraint = {"garch_stationary": 1, "tb_supercritical": 2}.get(spec.get("constraint"), 0)
    m.x0 = float(spec.get("x0", 0.0))
    m.t_end = float(spec.get("t_end", 0.0))
    m.steps = int(spec.get("steps", 0))
    m.n_obs = int(spec.get("n_obs", 0))
    m.noise_sd = float(spec.get("noise_sd", 0.0))
    m.n_cells = int(spec.get("n_cells", 0))
    return m


def threads() -> int:
    """OpenMP threads the oracle will use."""
    return int(_load().or_max_threads())


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    _load().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def stream_block(seed: int, draw: int, block: int, purpose: int) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    _load().or_stream_block(seed, draw, block, purpose, out)
    return out


def uniform(word: int) -> float:
    return float(_load().or_uniform(word))


def angle_uniform(word_i: int, word3: int, i: int) -> float:
    """Angle uniform of Box-Muller pair i of a path or cell block (words i and 3)."""
    return float(_load().or_angle_uniform(word_i, word3, i))


def box_muller(w0: int, w1: int) -> tuple[float, float]:
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    _load().or_box_muller(w0, w1, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def path_normal(seed: int, draw: int, n: int) -> float:
    """Normal n of a draw's path stream: block n // 6, pair (n % 6) // 2."""
    return float(_load().or_path_normal(seed, draw, n))


def cell_normal(seed: int, draw: int, cell: int, n: int) -> float:
    """Normal n of cell `cell` of a draw (multi-cell models)."""
    return float(_load().or_cell_normal(seed, draw, cell, n))


def toggle_cells(spec: Mapping, theta, seed: int, draw: int) -> dict:
    """Final levels u, v and measurement y of every cell of one toggle-switch
    draw at the given theta (cell order)."""
    m = _model(spec)
    c = m.n_cells
    u, v, y = (np.zeros(c, np.float64) for _ in range(3))
    rc = _load().or_toggle_cells(ctypes.byref(m), np.ascontiguousarray(theta, np.float64), seed,
                                 draw, u, v, y)
    if rc != 0:
        raise ValueError("oracle: not a valid toggle-switch model")
    return {"u": u, "v": v, "y": y}


def n_summaries(spec: Mapping) -> int:
    return int(_load().or_n_summaries(ctypes.byref(_model(spec))))


def prior_draw(spec: Mapping, seed: int, draw: int) -> tuple[np.ndarray, int]:
    m = _model(spec)
    theta = np.zeros(m.n_params, np.float64)
    attempts = _load().or_prior_draw(ctypes.byref(m), seed, draw, theta)
    return theta, int(attempts)


def simulate(spec: Mapping, seed: int, first: int, n: int, y_obs=None) -> dict:
    """Per-draw theta, summaries, mean statistic, distance and prior attempts."""
    m = _model(spec)
    ns = n_summaries(spec)
    theta = np.zeros((n, m.n_params), np.float64)
    summ = np.zeros((n, ns), np.float64)
    stat = np.zeros(n, np.float64)
    dist = np.zeros(n, np.float64)
    att = np.zeros(n, np.int32)
    y = None
    if y_obs is not None:
        y = np.ascontiguousarray(y_obs, np.float64)
        assert y.shape == (ns,)
    rc = _load().or_simulate(ctypes.byref(m), seed, first, n,
                             y.ctypes.data if y is not None else None,
                             theta, summ, stat, dist, att)
    _check(rc, "invalid model")
    return {"theta": theta, "summ": summ, "stat": stat, "dist": dist, "attempts": att}


def top_count(frac: float, n: int) -> int:
    return int(_load().or_top_count(frac, n))


def abc(spec: Mapping, y_obs, seed: int, first: int, n: int, mode: int, eps_or_frac: float,
        capacity: int | None = None) -> dict:
    m = _model(spec)
    cap = n if capacity is None else capacity
    idx = np.zeros(max(cap, 1), np.uint64)
    th = np.zeros((max(cap, 1), m.n_params), np.float64)
    d = np.zeros(max(cap, 1), np.float64)
    nacc = ctypes.c_uint64()
    eps = ctypes.c_double()
    mean = np.zeros(MAX_PARAMS, np.float64)
    var = np.zeros(MAX_PARAMS, np.float64)
    rc = _load().or_abc(ctypes.byref(m), np.ascontiguousarray(y_obs, np.float64), seed, first, n,
                        mode, eps_or_frac, cap, idx, th, d, ctypes.byref(nacc), ctypes.byref(eps),
                        mean, var)
    _check(rc, "invalid input")
    k = min(int(nacc.value), cap)
    return {"idx": idx[:k], "theta": th[:k], "dist": d[:k], "n_accepted": int(nacc.value),
            "eps_used": float(eps.value), "mean": mean[: m.n_params], "var": var[: m.n_params],
            "truncated": rc == 1}


def pvalue(spec: Mapping, lambda_param: int, lambda_family: str, lambdas, seed: int, first: int,
           n: int, t_obs: float) -> dict:
    m = _model(spec)
    lam = np.ascontiguousarray(lambdas, np.float64)
    counts = np.zeros(len(lam), np.uint64)
    p = np.zeros(len(lam), np.float64)
    rc = _load().or_pvalue(ctypes.byref(m), lambda_param, _FAMILY[lambda_family], lam, len(lam),
                           seed, first, n, t_obs, counts, p)
    _check(rc, "invalid input")
    return {"count_ge": counts, "pvalue": p}


def summary_tally(spec: Mapping, seed: int, first: int, n: int, obs_summ) -> np.ndarray:
    m = _model(spec)
    ns = n_summaries(spec)
    counts = np.zeros(ns, np.uint64)
    rc = _load().or_summary_tally(ctypes.byref(m), seed, first, n,
                                  np.ascontiguousarray(obs_summ, np.float64), counts)
    _check(rc, "invalid input")
    return counts


def logistic_path(spec: Mapping, theta, seed: int, draw: int) -> np.ndarray:
    m = _model(spec)
    path = np.zeros(m.steps, np.float64)
    rc = _load().or_logistic_path(ctypes.byref(m), np.ascontiguousarray(theta, np.float64), seed,
                                  draw, path)
    if rc != 0:
        raise ValueError("oracle: not a logistic model")
    return path


def garch_series(spec: Mapping, theta, seed: int, draw: int) -> np.ndarray:
    m = _model(spec)
    r = np.zeros(m.steps, np.float64)
    rc = _load().or_garch_series(ctypes.byref(m), np.ascontiguousarray(theta, np.float64), seed,
                                 draw, r)
    if rc != 0:
        raise ValueError("oracle: not a GARCH model")
    return r


def garch_summaries(r) -> np.ndarray:
    r = np.ascontiguousarray(r, np.float64)
    s = np.zeros(GARCH_NSUMM, np.float64)
    _load().or_garch_summaries(r, len(r), s)
    return s


def garch_bar_scales(spec: Mapping, seed: int, draws) -> np.ndarray:
    """Per draw and GARCH summary, the magnitude an error bar is relative to
    (test infrastructure, not part of the method).  Variance and kurtosis
    are sums of non-negative terms: their own value.  The mean and the
    skewness are signed sums that can lie arbitrarily close to 0, where the
    rounding of the normals to FP32 alone moves them by far more than a fixed
    fraction of their value: for them the scale is the same sum over
    absolute terms, (1/L) sum |r_t| for the mean and
    (1/L) sum |r_t - rbar|^3 / m2^1.5 for the skewness (componentwise
    relative error).  The squared-return ACFs are normalised: scale 1."""
    draws = np.asarray(list(draws), np.int64)
    out = np.zeros((len(draws), GARCH_NSUMM), np.float64)
    for q, i in enumerate(draws):
        th, _ = prior_draw(spec, seed, int(i))
        r = garch_series(spec, th, seed, int(i))
        s = garch_summaries(r)
        d = r - r.mean()
        m2 = np.mean(d * d)
        out[q, 0] = np.mean(np.abs(r))
        out[q, 1] = abs(s[1])
        out[q, 2] = np.mean(np.abs(d) ** 3) / m2 ** 1.5
        out[q, 3] = abs(s[3])
        out[q, 4:] = 1.0
    return out


def distance(x, y) -> float:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    return float(_load().or_distance(x, y, len(x)))


def _bioassay(spec: Mapping) -> _Bioassay:
    b = _Bioassay()
    b.n_groups = len(spec["dose"])
    for i, (n, x) in enumerate(zip(spec["n_trials"], spec["dose"])):
        b.n_trials[i] = int(n)
        b.dose[i] = float(x)
    return b


def _smc(cfg: Mapping) -> _SmcConfig:
    c = _SmcConfig()
    c.n_particles = int(cfg["n_particles"])
    c.max_mcmc = int(cfg["max_mcmc"])
    c.max_steps = int(cfg["max_steps"])
    c.bisect_iters = int(cfg["bisect_iters"])
    c.c = float(cfg["c"])
    c.h = float(cfg["h"])
    return c


def bio_simulate(spec: Mapping, lam, seed: int, data_id: int, purpose: int) -> tuple[np.ndarray, np.ndarray]:
    """One data set D ~ p(D | lambda): (y per group, theta)."""
    y = np.zeros(len(spec["dose"]), np.int32)
    th = np.zeros(2, np.float64)
    _load().or_bio_simulate(ctypes.byref(_bioassay(spec)), np.ascontiguousarray(lam, np.float64),
                            seed, data_id, purpose, y, th)
    return y, th


def bio_loglik(spec: Mapping, y, b0: float, b1: float) -> float:
    return float(_load().or_bio_loglik(ctypes.byref(_bioassay(spec)),
                                       np.ascontiguousarray(y, np.int32), b0, b1))


def bio_logprior(lam, b0: float, b1: float) -> float:
    return float(_load().or_bio_logprior(np.ascontiguousarray(lam, np.float64), b0, b1))


def smc_log_evidence(spec: Mapping, y, lam, cfg: Mapping, seed: int, run: int) -> dict:
    """Alg. 3 for log p(D | lambda); trace rows (t_n, delta_n, p_acc_n, R_n)."""
    c = _smc(cfg)
    trace = np.zeros((c.max_steps, 4), np.float64)
    n = ctypes.c_int32()
    lz = _load().or_smc_log_evidence(ctypes.byref(_bioassay(spec)), np.ascontiguousarray(y, np.int32),
                                     np.ascontiguousarray(lam, np.float64), ctypes.byref(c), seed,
                                     run, ctypes.byref(n), trace.ctypes.data)
    return {"log_z": float(lz), "n_steps": int(n.value), "trace": trace[: n.value]}


def wip_test(spec: Mapping, lambdas, n_data: int, cfg: Mapping, seed: int, alpha: float) -> dict:
    """Alg. 2: log evidences, p-values and alpha cut-offs per lambda (row 0 =
    the base prior)."""
    lam = np.ascontiguousarray(lambdas, np.float64).reshape(-1, 2)
    k = lam.shape[0]
    lz0 = np.zeros((k, n_data), np.float64)
    lzk = np.zeros((k, n_data), np.float64)
    pv = np.zeros((k, n_data), np.float64)
    gamma = np.zeros(k, np.float64)
    rc = _load().or_wip_test(ctypes.byref(_bioassay(spec)), lam, k, n_data, ctypes.byref(_smc(cfg)),
                             seed, alpha, lz0, lzk, pv, gamma)
    if rc != 0:
        raise ValueError("oracle: invalid weak-informativity input")
    return {"log_z0": lz0, "log_zk": lzk, "pvalues": pv, "gamma": gamma}


def smc_temper(ll, t: float, step: int, cfg: Mapping) -> float:
    """Tempering increment of one SMC step (the ESS = N_p / 2 condition)."""
    ll = np.ascontiguousarray(ll, np.float64)
    return float(_load().or_smc_temper(ll, len(ll), t, step, ctypes.byref(_smc(cfg))))


def smc_resample(w, seed: int, run: int, step: int) -> np.ndarray:
    """Ancestors of a multinomial resampling step with weights w (max 1)."""
    w = np.ascontiguousarray(w, np.float64)
    anc = np.zeros(len(w), np.int32)
    _load().or_smc_resample(w, len(w), seed, run, step, anc)
    return anc


def smc_proposal(b0, b1, h: float) -> np.ndarray:
    """(l11, l21, l22): the Cholesky factor of h^2 times the sample covariance."""
    out = np.zeros(3, np.float64)
    b0 = np.ascontiguousarray(b0, np.float64)
    _load().or_smc_proposal(b0, np.ascontiguousarray(b1, np.float64), len(b0), h, out)
    return out


def smc_moves(accepted: int, n_particles: int, cfg: Mapping) -> int:
    return int(_load().or_smc_moves(accepted, n_particles, ctypes.byref(_smc(cfg))))


def gamma_p(a: float, x: float) -> float:
    """Regularised lower incomplete gamma function P(a, x)."""
    return float(_load().or_gamma_p(a, x))


def gamma_q(a: float, x: float) -> float:
    """Q(a, x) = 1 - P(a, x), the upper regularised incomplete gamma function."""
    return float(_load().or_gamma_q(a, x))


def bege_cdf(u: float, p: float, n: float, sp: float, sn: float, n_omega: int = 100) -> float:
    return float(_load().or_bege_cdf(u, p, n, sp, sn, n_omega))


def bege_density(u: float, p: float, n: float, sp: float, sn: float, n_omega: int = 100) -> float:
    return float(_load().or_bege_density(u, p, n, sp, sn, n_omega))


def bege_density_q(u: float, p: float, n: float, sp: float, sn: float, n_omega: int = 100) -> float:
    """The central difference of bege_density with every operation in quad
    precision (the FP64 density uses it where its two sums cancel)."""
    return float(_load().or_bege_density_q(u, p, n, sp, sn, n_omega))


def bege_loglik(theta, r, n_omega: int = 100) -> dict:
    """log L(theta; r_0..r_T) and the T per-step log densities."""
    th = np.ascontiguousarray(theta, np.float64)
    rr = np.ascontiguousarray(r, np.float64)
    T = len(rr) - 1
    ld = np.zeros(T, np.float64)
    out = ctypes.c_double()
    _load().or_bege_loglik(th, rr, T, n_omega, ld.ctypes.data, ctypes.byref(out))
    return {"loglik": float(out.value), "logdens": ld}


def bege_loglik_batch(thetas, r, n_omega: int = 100, with_logdens: bool = False):
    """log L of every row (OpenMP over rows); with_logdens: (log L, log f
    of every (row, step)) instead."""
    th = np.ascontiguousarray(thetas, np.float64).reshape(-1, 11)
    rr = np.ascontiguousarray(r, np.float64)
    out = np.zeros(th.shape[0], np.float64)
    ld = np.zeros((th.shape[0], len(rr) - 1), np.float64) if with_logdens else None
    _load().or_bege_loglik_batch(th, th.shape[0], rr, len(rr) - 1, n_omega, out,
                                 None if ld is None else ld.ctypes.data)
    return (out, ld) if with_logdens else out


def bege_simulate(theta, T: int, seed: int) -> np.ndarray:
    """A synthetic BEGE return series r_0..r_T at theta."""
    r = np.zeros(T + 1, np.float64)
    rc = _load().or_bege_simulate(np.ascontiguousarray(theta, np.float64), T, seed, r)
    if rc != 0:
        raise ValueError("oracle: a BEGE shape became non-positive")
    return r


# ---- tuberculosis transmission (App. B) -------------------------------------

def tb_select(counts, m: int) -> int:
    """Slot of case m in slot order (the lookup over genotype weights)."""
    x = np.ascontiguousarray(counts, np.uint32)
    return int(_load().or_tb_select(x, len(x), m))


def tb_lowest_empty(counts) -> int:
    x = np.ascontiguousarray(counts, np.uint32)
    return int(_load().or_tb_lowest_empty(x, len(x)))


def tb_thresholds(theta) -> tuple[int, int]:
    tb, td = ctypes.c_uint64(), ctypes.c_uint64()
    _load().or_tb_thresholds(np.ascontiguousarray(theta, np.float64), ctypes.byref(tb), ctypes.byref(td))
    return tb.value, td.value


def tb_run(theta, n_stop: int, seed: int, draw: int, max_events: int = 2**31 - 1,
           x0: float = 1.0) -> dict:
    """One run at theta = (alpha, delta, tau): status, events, final N and
    the final case counts per genotype slot."""
    X = np.zeros(n_stop, np.uint32)
    ev, N = ctypes.c_uint64(), ctypes.c_uint64()
    st = _load().or_tb_run(np.ascontiguousarray(theta, np.float64), n_stop, x0, max_events, seed, draw,
                           X, ctypes.byref(ev), ctypes.byref(N))
    return {"status": int(st), "events": int(ev.value), "n": int(N.value), "counts": X}


def tb_summaries(counts, n_sample: int, seed: int, draw: int) -> np.ndarray:
    X = np.array(counts, np.uint32)
    Y = np.zeros_like(X)
    out = np.zeros(2, np.float64)
    _load().or_tb_summaries(X, Y, len(X), int(X.sum()), n_sample, seed, draw, out)
    return out


def tb_simulate(spec: Mapping, seed: int, first: int, n: int) -> dict:
    """Per draw: theta, status, events, final N, summaries (g/n_s, H)."""
    m = _model(spec)
    theta = np.zeros((n, 3), np.float64)
    status = np.zeros(n, np.int32)
    events = np.zeros(n, np.uint64)
    nf = np.zeros(n, np.uint64)
    summ = np.zeros((n, 2), np.float64)
    rc = _load().or_tb_simulate(ctypes.byref(m), seed, first, n, theta, status, events, nf, summ)
    _check(rc, "invalid tuberculosis model")
    return {"theta": theta, "status": status, "events": events, "n": nf, "summ": summ}
