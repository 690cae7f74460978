"""ctypes binding of libpps.so (include/pps.h): argument marshalling only.

Every function here has the name of the C entry point it wraps; each step of
the sampler runs in the library's HIP kernels.  Device buffers are torch
tensors on the current HIP device (their ``data_ptr()`` is passed through),
and ``stream`` defaults to torch's current stream.  There is no fallback: if
the library is missing, loading fails with an error that says so.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Mapping, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpps.so")

PPS_OK, PPS_PENDING = 0, 1
PPS_EINVAL, PPS_ENOMEM, PPS_EDEVICE, PPS_EBUSY, PPS_ENOTFOUND, PPS_ETRUNC = -1, -2, -3, -4, -5, -6
PPS_UNIFORM, PPS_NORMAL, PPS_LOGNORMAL, PPS_POINT = 0, 1, 2, 3
PPS_LOGISTIC_SDE, PPS_GARCH11, PPS_NORMAL_MEAN = 0, 1, 2
PPS_NO_CONSTRAINT, PPS_GARCH_STATIONARY = 0, 1
PPS_EPS_FIXED, PPS_EPS_TOP_FRACTION = 0, 1
PPS_MAX_PARAMS, PPS_MAX_OBS, PPS_GARCH_NSUMM = 4, 64, 14

FAMILY = {"uniform": PPS_UNIFORM, "normal": PPS_NORMAL, "lognormal": PPS_LOGNORMAL,
          "point": PPS_POINT}
MODEL = {"logistic": PPS_LOGISTIC_SDE, "garch11": PPS_GARCH11, "normal_mean": PPS_NORMAL_MEAN}


class PPSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class pps_prior(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double)]


class pps_model(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("n_params", ctypes.c_int32),
        ("prior", pps_prior * PPS_MAX_PARAMS),
        ("constraint", ctypes.c_int32),
        ("x0", ctypes.c_double),
        ("t_end", ctypes.c_double),
        ("steps", ctypes.c_int32),
        ("n_obs", ctypes.c_int32),
        ("noise_sd", ctypes.c_double),
    ]


class pps_sampling(ctypes.Structure):
    _fields_ = [("n_draws", ctypes.c_uint64), ("first_draw", ctypes.c_uint64),
                ("seed", ctypes.c_uint64)]


class pps_abc_stats(ctypes.Structure):
    _fields_ = [("n_accepted", ctypes.c_uint64), ("eps_used", ctypes.c_double),
                ("mean", ctypes.c_double * PPS_MAX_PARAMS), ("var", ctypes.c_double * PPS_MAX_PARAMS)]


_lib = None


def lib():
    """The loaded libpps.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1902_09046_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32, f64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        mp, sp = ctypes.POINTER(pps_model), ctypes.POINTER(pps_sampling)
        L.pps_philox.argtypes = [u64, u64, u64, ctypes.c_uint32, ctypes.c_uint32, vp, vp]
        L.pps_normals.argtypes = [u64, u64, u64, ctypes.c_uint32, vp, vp]
        L.pps_simulate.argtypes = [mp, sp, vp, vp, vp, vp, vp, vp]
        L.pps_n_summaries.argtypes = [mp]
        L.abc_sample.argtypes = [mp, vp, sp, i32, f64, u64, vp, vp, vp,
                                 ctypes.POINTER(pps_abc_stats), vp]
        L.prior_pred_pvalue.argtypes = [mp, i32, i32, vp, i32, sp, f64, vp, vp, vp]
        L.pps_summary_tally.argtypes = [mp, sp, vp, vp, vp]
        L.pps_strerror.argtypes = [i32]
        L.pps_strerror.restype = ctypes.c_char_p
        L.pps_last_error.restype = ctypes.c_char_p
        L.pps_version.restype = ctypes.c_char_p
        L.pps_set_timing.argtypes = [ctypes.c_int]
        L.pps_set_timing.restype = ctypes.c_int
        L.pps_last_kernel_ms.restype = ctypes.c_double
        L.pps_set_block_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.pps_set_block_size.restype = ctypes.c_int
        L.pps_get_block_size.argtypes = [ctypes.c_int]
        L.pps_get_block_size.restype = ctypes.c_int
        L.pps_set_launch_shape.argtypes = [ctypes.c_int] * 4
        L.pps_set_launch_shape.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.pps_get_launch_shape.argtypes = [ctypes.c_int, ip, ip, ip]
        L.pps_get_launch_shape.restype = ctypes.c_int
        for name in ("pps_philox", "pps_normals", "pps_simulate", "pps_n_summaries", "abc_sample",
                     "prior_pred_pvalue", "pps_summary_tally"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, allow=(PPS_OK,)) -> int:
    if status not in allow:
        msg = lib().pps_last_error().decode() or lib().pps_strerror(status).decode()
        raise PPSError(status, msg)
    return status


def make_model(spec: Mapping) -> pps_model:
    """pps_model from a workload spec dict (see pps_workloads)."""
    m = pps_model()
    m.model = MODEL[spec["model"]]
    priors = spec["priors"]
    m.n_params = len(priors)
    for j, (fam, a, b) in enumerate(priors):
        m.prior[j].family = FAMILY[fam]
        m.prior[j].a = float(a)
        m.prior[j].b = float(b)
    m.constraint = PPS_GARCH_STATIONARY if spec.get("constraint") == "garch_stationary" else 0
    m.x0 = float(spec.get("x0", 0.0))
    m.t_end = float(spec.get("t_end", 0.0))
    m.steps = int(spec.get("steps", 0))
    m.n_obs = int(spec.get("n_obs", 0))
    m.noise_sd = float(spec.get("noise_sd", 0.0))
    return m


def make_sampling(n_draws: int, first_draw: int = 0, seed: int = 1) -> pps_sampling:
    return pps_sampling(n_draws, first_draw, seed)


def _model_arg(model) -> pps_model:
    return model if isinstance(model, pps_model) else make_model(model)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _host_f64(values) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(values, dtype=np.float64))


def pps_version() -> str:
    return lib().pps_version().decode()


def pps_set_timing(enable: bool) -> None:
    _check(lib().pps_set_timing(1 if enable else 0))


def pps_last_kernel_ms() -> float:
    return float(lib().pps_last_kernel_ms())


def pps_set_block_size(model_class: int, block: int) -> None:
    _check(lib().pps_set_block_size(model_class, block))


def pps_get_block_size(model_class: int) -> int:
    return _check_count(lib().pps_get_block_size(model_class))


def pps_set_launch_shape(model_class: int, block: int, draws_per_lane: int = 1,
                         unroll: int = 1) -> None:
    _check(lib().pps_set_launch_shape(model_class, block, draws_per_lane, unroll))


def pps_get_launch_shape(model_class: int) -> tuple[int, int, int]:
    b, d, u = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().pps_get_launch_shape(model_class, ctypes.byref(b), ctypes.byref(d), ctypes.byref(u)))
    return b.value, d.value, u.value


PATH_SHAPES = [(b, d, u) for b in (64, 128, 256) for d in (1, 2) for u in (1, 2)]
GARCH_SHAPES = [(b, 1, 1) for b in (64, 128, 256)]


def pps_n_summaries(model) -> int:
    return _check_count(lib().pps_n_summaries(ctypes.byref(_model_arg(model))))


def _check_count(v: int) -> int:
    if v < 0:
        _check(v)
    return v


def pps_philox(seed: int, first_draw: int, n: int, block: int, purpose: int, out, stream=None):
    _check(lib().pps_philox(seed, first_draw, n, block, purpose, _ptr(out), _stream(stream)))


def pps_normals(seed: int, first_draw: int, n: int, m: int, out, stream=None):
    _check(lib().pps_normals(seed, first_draw, n, m, _ptr(out), _stream(stream)))


def pps_simulate(model, sampling: pps_sampling, y_obs, theta, summ, stat, dist, stream=None):
    y = None if y_obs is None else _host_f64(y_obs)
    _check(lib().pps_simulate(ctypes.byref(_model_arg(model)), ctypes.byref(sampling),
                              None if y is None else y.ctypes.data, _ptr(theta), _ptr(summ),
                              _ptr(stat), _ptr(dist), _stream(stream)))


def abc_sample(model, y_obs, sampling: pps_sampling, eps_mode: int, eps_or_frac: float,
               capacity: int, acc_idx, acc_theta, acc_dist, stream=None) -> tuple[int, dict]:
    """Returns (status, stats); status is PPS_OK or PPS_ETRUNC."""
    y = _host_f64(y_obs)
    st = pps_abc_stats()
    rc = lib().abc_sample(ctypes.byref(_model_arg(model)), y.ctypes.data, ctypes.byref(sampling),
                          eps_mode, eps_or_frac, capacity, _ptr(acc_idx), _ptr(acc_theta),
                          _ptr(acc_dist), ctypes.byref(st), _stream(stream))
    _check(rc, allow=(PPS_OK, PPS_ETRUNC))
    return rc, {"n_accepted": int(st.n_accepted), "eps_used": float(st.eps_used),
                "mean": np.array(st.mean[:]), "var": np.array(st.var[:])}


def prior_pred_pvalue(model, lambda_param: int, lambda_family: int, lambdas: Sequence[float],
                      sampling: pps_sampling, t_obs: float, stream=None) -> tuple[np.ndarray, np.ndarray]:
    lam = _host_f64(lambdas)
    counts = np.zeros(len(lam), np.uint64)
    p = np.zeros(len(lam), np.float64)
    _check(lib().prior_pred_pvalue(ctypes.byref(_model_arg(model)), lambda_param, lambda_family,
                                   lam.ctypes.data, len(lam), ctypes.byref(sampling), t_obs,
                                   counts.ctypes.data, p.ctypes.data, _stream(stream)))
    return counts, p


def pps_summary_tally(model, sampling: pps_sampling, obs_summ, stream=None) -> np.ndarray:
    obs = _host_f64(obs_summ)
    counts = np.zeros(len(obs), np.uint64)
    _check(lib().pps_summary_tally(ctypes.byref(_model_arg(model)), ctypes.byref(sampling),
                                   obs.ctypes.data, counts.ctypes.data, _stream(stream)))
    return counts


# --------------------------------------------------------------------------
# Conveniences that allocate the output tensors (still marshalling only).
# --------------------------------------------------------------------------
def simulate(spec: Mapping, seed: int, first: int, n: int, y_obs=None, device="cuda"):
    """Per-draw theta (n_params, n), summaries (ns, n), stat (n), dist (n)."""
    import torch
    model = make_model(spec)
    ns = pps_n_summaries(model)
    theta = torch.empty((model.n_params, n), dtype=torch.float32, device=device)
    summ = torch.empty((ns, n), dtype=torch.float32, device=device)
    garch = model.model == PPS_GARCH11
    stat = None if garch else torch.empty(n, dtype=torch.float32, device=device)
    dist = None if (garch or y_obs is None) else torch.empty(n, dtype=torch.float32, device=device)
    pps_simulate(model, make_sampling(n, first, seed), y_obs, theta, summ, stat, dist)
    return {"theta": theta, "summ": summ, "stat": stat, "dist": dist}


def abc(spec: Mapping, y_obs, seed: int, first: int, n: int, eps_mode: int, eps_or_frac: float,
        capacity: int | None = None, device="cuda"):
    import torch
    model = make_model(spec)
    if capacity is None:
        capacity = n if eps_mode == PPS_EPS_FIXED else int(math.ceil(eps_or_frac * n)) + 1
    idx = torch.empty(max(capacity, 1), dtype=torch.int64, device=device)
    th = torch.empty((model.n_params, max(capacity, 1)), dtype=torch.float32, device=device)
    d = torch.empty(max(capacity, 1), dtype=torch.float32, device=device)
    rc, st = abc_sample(model, y_obs, make_sampling(n, first, seed), eps_mode, eps_or_frac,
                        capacity, idx, th, d)
    k = min(st["n_accepted"], capacity)
    st.update({"status": rc, "idx": idx[:k], "theta": th[:, :k], "dist": d[:k]})
    return st
