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
PPS_LOGISTIC_SDE, PPS_GARCH11, PPS_NORMAL_MEAN, PPS_TOGGLE_SWITCH, PPS_TB = 0, 1, 2, 3, 4
PPS_NO_CONSTRAINT, PPS_GARCH_STATIONARY, PPS_TB_SUPERCRITICAL = 0, 1, 2
PPS_EPS_FIXED, PPS_EPS_TOP_FRACTION = 0, 1
PPS_MAX_PARAMS, PPS_MAX_OBS, PPS_GARCH_NSUMM, PPS_TSW_MAX_CELLS = 8, 64, 14, 8192
PPS_TB_MAX_POP, PPS_TB_MAX_SAMPLE = 16384, 1024
PPS_NOALLOC_MAX_DRAWS = 1 << 22
# kernel classes (pps_set_launch_shape)
CLASS_PATH, CLASS_GARCH, CLASS_GROUP, CLASS_CELLS, CLASS_GILLESPIE = 0, 1, 2, 3, 4

FAMILY = {"uniform": PPS_UNIFORM, "normal": PPS_NORMAL, "lognormal": PPS_LOGNORMAL,
          "point": PPS_POINT}
MODEL = {"logistic": PPS_LOGISTIC_SDE, "garch11": PPS_GARCH11, "normal_mean": PPS_NORMAL_MEAN,
         "toggle_switch": PPS_TOGGLE_SWITCH, "tb": PPS_TB}


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
        ("n_cells", ctypes.c_int32),
    ]


class pps_sampling(ctypes.Structure):
    _fields_ = [("n_draws", ctypes.c_uint64), ("first_draw", ctypes.c_uint64),
                ("seed", ctypes.c_uint64)]


class pps_abc_stats(ctypes.Structure):
    _fields_ = [("n_accepted", ctypes.c_uint64), ("eps_used", ctypes.c_double),
                ("mean", ctypes.c_double * PPS_MAX_PARAMS), ("var", ctypes.c_double * PPS_MAX_PARAMS)]


PPS_JOB_ABC, PPS_JOB_PVALUE = 0, 1
PPS_POLICY_BATCHED, PPS_POLICY_PLAIN = 0, 1


class pps_job(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("model", pps_model),
        ("sampling", pps_sampling),
        ("y_obs", ctypes.c_double * PPS_MAX_OBS),
        ("eps_mode", ctypes.c_int32),
        ("eps_or_frac", ctypes.c_double),
        ("capacity", ctypes.c_uint64),
        ("lambda_param", ctypes.c_int32),
        ("lambda_family", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("t_obs", ctypes.c_double),
    ]


class pps_job_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("kind", ctypes.c_int32),
        ("abc", pps_abc_stats),
        ("count_ge", ctypes.c_uint64),
        ("pvalue", ctypes.c_double),
        ("acc_idx", ctypes.c_void_p),
        ("acc_theta", ctypes.c_void_p),
        ("acc_dist", ctypes.c_void_p),
        ("n_records", ctypes.c_uint64),
        ("record_stride", ctypes.c_uint64),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class pps_server_config(ctypes.Structure):
    _fields_ = [
        ("arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_uint64),
        ("max_active", ctypes.c_int32),
        ("queue_capacity", ctypes.c_int32),
        ("epoch_ms", ctypes.c_double),
        ("policy", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class pps_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("epochs", ctypes.c_uint64),
        ("queued", ctypes.c_uint64), ("active", ctypes.c_uint64), ("busy_s", ctypes.c_double),
        ("latency_p50_s", ctypes.c_double), ("latency_p99_s", ctypes.c_double),
    ]


class pps_tune_entry(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("draws_per_lane", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("ms", ctypes.c_double)]


class pps_tune_report(ctypes.Structure):
    _fields_ = [("model_class", ctypes.c_int32), ("n_entries", ctypes.c_int32),
                ("entries", pps_tune_entry * 16), ("best", ctypes.c_int32),
                ("from_cache", ctypes.c_int32)]


PPS_BIO_MAX_GROUPS, PPS_SMC_MAX_PARTICLES = 8, 1024


class pps_bioassay(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("n_trials", ctypes.c_int32 * PPS_BIO_MAX_GROUPS),
                ("dose", ctypes.c_double * PPS_BIO_MAX_GROUPS)]


class pps_smc_config(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int32), ("max_mcmc", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("bisect_iters", ctypes.c_int32),
                ("c", ctypes.c_double), ("h", ctypes.c_double)]


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
        L.abc_sample_noalloc.argtypes = [mp, vp, sp, i32, f64, u64, vp, vp, vp,
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
        L.pps_last_finalize_ms.restype = ctypes.c_double
        L.pps_set_block_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.pps_set_block_size.restype = ctypes.c_int
        L.pps_get_block_size.argtypes = [ctypes.c_int]
        L.pps_get_block_size.restype = ctypes.c_int
        L.pps_set_launch_shape.argtypes = [ctypes.c_int] * 4
        L.pps_set_launch_shape.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.pps_get_launch_shape.argtypes = [ctypes.c_int, ip, ip, ip]
        L.pps_get_launch_shape.restype = ctypes.c_int
        jp, rp, cp = ctypes.POINTER(pps_job), ctypes.POINTER(pps_job_result), ctypes.POINTER(pps_server_config)
        L.pps_job_arena_bytes.argtypes = [jp]
        L.pps_job_arena_bytes.restype = ctypes.c_int64
        L.pps_run_batch.argtypes = [jp, ctypes.c_int, cp, rp]
        L.pps_server_create.argtypes = [cp, ctypes.POINTER(ctypes.c_void_p)]
        L.pps_submit.argtypes = [vp, jp, ctypes.POINTER(ctypes.c_uint64)]
        L.pps_poll.argtypes = [vp, u64, rp]
        L.pps_release.argtypes = [vp, u64]
        L.pps_server_stats_get.argtypes = [vp, ctypes.POINTER(pps_server_stats)]
        L.pps_server_destroy.argtypes = [vp]
        L.pps_server_inject_error.argtypes = [vp, u64, ctypes.c_int]
        L.pps_autotune.argtypes = [mp, u64, ctypes.c_int, ctypes.POINTER(pps_tune_report), vp]
        L.pps_autotune.restype = ctypes.c_int
        bp, scp = ctypes.POINTER(pps_bioassay), ctypes.POINTER(pps_smc_config)
        L.pps_smc_log_evidence.argtypes = [bp, vp, vp, u64, scp, u64, u64, vp, vp]
        L.pps_smc_log_evidence.restype = ctypes.c_int
        L.pps_wip_test.argtypes = [bp, vp, ctypes.c_int, u64, scp, u64, f64, vp, vp, vp, vp, vp]
        L.pps_wip_test.restype = ctypes.c_int
        L.pps_bege_loglik.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.pps_bege_loglik.restype = ctypes.c_int
        L.pps_tb_events.argtypes = [mp, sp, vp, vp, vp]
        L.pps_tb_events.restype = ctypes.c_int
        L.pps_bege_count_ops.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), vp]
        L.pps_bege_count_ops.restype = ctypes.c_int
        for name in ("pps_philox", "pps_normals", "pps_simulate", "pps_n_summaries", "abc_sample",
                     "abc_sample_noalloc",
                     "prior_pred_pvalue", "pps_summary_tally", "pps_run_batch", "pps_server_create",
                     "pps_submit", "pps_poll", "pps_release", "pps_server_stats_get",
                     "pps_server_destroy", "pps_server_inject_error"):
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
    m.constraint = {"garch_stationary": PPS_GARCH_STATIONARY,
                    "tb_supercritical": PPS_TB_SUPERCRITICAL}.get(spec.get("constraint"), 0)
    m.x0 = float(spec.get("x0", 0.0))
    m.t_end = float(spec.get("t_end", 0.0))
    m.steps = int(spec.get("steps", 0))
    m.n_obs = int(spec.get("n_obs", 0))
    m.noise_sd = float(spec.get("noise_sd", 0.0))
    m.n_cells = int(spec.get("n_cells", 0))
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


def pps_last_finalize_ms() -> float:
    return float(lib().pps_last_finalize_ms())


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
CELL_SHAPES = [(b, 1, 1) for b in (256, 512, 1024)]


def pps_autotune(model, n_draws: int, use_cache: bool = True, stream=None) -> dict:
    """Times the launch shapes of the model's class and keeps the fastest."""
    r = pps_tune_report()
    _check(lib().pps_autotune(ctypes.byref(_model_arg(model)), n_draws, 1 if use_cache else 0,
                              ctypes.byref(r), _stream(stream)))
    entries = [(e.block, e.draws_per_lane, e.unroll, e.ms) for e in r.entries[: r.n_entries]]
    best = entries[r.best][:3] if r.best >= 0 else None
    return {"model_class": r.model_class, "entries": entries, "best": best,
            "from_cache": bool(r.from_cache)}


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


def abc_sample_noalloc(model, y_obs, sampling: pps_sampling, eps_mode: int, eps_or_frac: float,
                       capacity: int, acc_idx, acc_theta, acc_dist, stream=None) -> tuple[int, dict]:
    """abc_sample with the library's static scratch (no allocation); the same
    return value as abc_sample."""
    y = _host_f64(y_obs)
    st = pps_abc_stats()
    rc = lib().abc_sample_noalloc(ctypes.byref(_model_arg(model)), y.ctypes.data,
                                  ctypes.byref(sampling), eps_mode, eps_or_frac, capacity,
                                  _ptr(acc_idx), _ptr(acc_theta), _ptr(acc_dist), ctypes.byref(st),
                                  _stream(stream))
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


# --------------------------------------------------------------------------
# Jobs, batches and serving.
# --------------------------------------------------------------------------
def make_abc_job(spec: Mapping, y_obs, sampling: pps_sampling, eps_mode: int, eps_or_frac: float,
                 capacity: int = 0) -> pps_job:
    j = pps_job()
    j.kind = PPS_JOB_ABC
    j.model = make_model(spec)
    j.sampling = sampling
    for k, v in enumerate(y_obs):
        j.y_obs[k] = float(v)
    j.eps_mode = eps_mode
    j.eps_or_frac = float(eps_or_frac)
    j.capacity = int(capacity)
    return j


def make_pvalue_job(spec: Mapping, lambda_param: int, lambda_family: int, lam: float,
                    sampling: pps_sampling, t_obs: float) -> pps_job:
    j = pps_job()
    j.kind = PPS_JOB_PVALUE
    j.model = make_model(spec)
    j.sampling = sampling
    j.lambda_param = lambda_param
    j.lambda_family = lambda_family
    j.lambda_ = float(lam)
    j.t_obs = float(t_obs)
    return j


def make_server_config(arena, arena_bytes: int | None = None, max_active: int = 256,
                       queue_capacity: int = 0, epoch_ms: float = 4.0,
                       policy: int = PPS_POLICY_BATCHED, stream=None) -> pps_server_config:
    c = pps_server_config()
    c.arena = int(arena.data_ptr())
    c.arena_bytes = int(arena_bytes if arena_bytes is not None else arena.numel() * arena.element_size())
    c.max_active = max_active
    c.queue_capacity = queue_capacity
    c.epoch_ms = epoch_ms
    c.policy = policy
    c.stream = None if stream is None else int(stream)
    return c


def pps_job_arena_bytes(job: pps_job) -> int:
    return _check_count(lib().pps_job_arena_bytes(ctypes.byref(job)))


def pps_run_batch(jobs, config: pps_server_config):
    arr = (pps_job * len(jobs))(*jobs)
    res = (pps_job_result * len(jobs))()
    _check(lib().pps_run_batch(arr, len(jobs), ctypes.byref(config), res))
    return list(res)


class Server:
    """pps_server_create / pps_submit / pps_poll / pps_release / pps_server_destroy."""

    def __init__(self, config: pps_server_config):
        self._cfg = config
        h = ctypes.c_void_p()
        _check(lib().pps_server_create(ctypes.byref(config), ctypes.byref(h)))
        self._h = h

    def submit(self, job: pps_job) -> int:
        jid = ctypes.c_uint64()
        _check(lib().pps_submit(self._h, ctypes.byref(job), ctypes.byref(jid)))
        return int(jid.value)

    def try_submit(self, job: pps_job):
        """Returns the job id, or None when the queue is full."""
        jid = ctypes.c_uint64()
        rc = lib().pps_submit(self._h, ctypes.byref(job), ctypes.byref(jid))
        if rc == PPS_EBUSY:
            return None
        _check(rc)
        return int(jid.value)

    def poll(self, job_id: int):
        """(status, result): status PPS_PENDING while running."""
        r = pps_job_result()
        rc = lib().pps_poll(self._h, job_id, ctypes.byref(r))
        if rc == PPS_ENOTFOUND:
            _check(rc)
        return rc, r

    def release(self, job_id: int) -> int:
        return lib().pps_release(self._h, job_id)

    def stats(self) -> pps_server_stats:
        s = pps_server_stats()
        _check(lib().pps_server_stats_get(self._h, ctypes.byref(s)))
        return s

    def inject_error(self, after_epochs: int, status: int) -> None:
        """Test hook: epochs harvested after the first `after_epochs` report
        `status` (< 0) and the server stops as after a device error."""
        _check(lib().pps_server_inject_error(self._h, after_epochs, status))

    def close(self):
        if self._h:
            _check(lib().pps_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def records(result: pps_job_result, arena, n_params: int):
    """A finished ABC job's records (index, theta (n_params, n), dist) as
    numpy arrays, read from the arena tensor the results point into."""
    n = int(result.n_records)
    base = int(arena.data_ptr())
    raw = arena.view(-1).view(__import__("torch").uint8)

    def span(ptr, nbytes):
        off = int(ptr) - base
        return raw[off:off + nbytes]

    if n == 0:
        return np.zeros(0, np.uint64), np.zeros((n_params, 0), np.float32), np.zeros(0, np.float32)
    stride = int(result.record_stride)
    idx = span(result.acc_idx, 8 * n).cpu().numpy().view(np.uint64).copy()
    th = np.stack([span(result.acc_theta + 4 * j * stride, 4 * n).cpu().numpy().view(np.float32)
                   for j in range(n_params)])
    d = span(result.acc_dist, 4 * n).cpu().numpy().view(np.float32).copy()
    return idx, th, d



# --------------------------------------------------------------------------
# Weak-informativity test (Sec. 4.1): SMC evidence (Alg. 3) and Alg. 2.
# --------------------------------------------------------------------------
def make_bioassay(spec: Mapping) -> pps_bioassay:
    """pps_bioassay from {"n_trials": [...], "dose": [...]}."""
    b = pps_bioassay()
    b.n_groups = len(spec["dose"])
    for i, (n, x) in enumerate(zip(spec["n_trials"], spec["dose"])):
        b.n_trials[i] = int(n)
        b.dose[i] = float(x)
    return b


def make_smc_config(cfg: Mapping) -> pps_smc_config:
    c = pps_smc_config()
    c.n_particles = int(cfg["n_particles"])
    c.max_mcmc = int(cfg["max_mcmc"])
    c.max_steps = int(cfg["max_steps"])
    c.bisect_iters = int(cfg["bisect_iters"])
    c.c = float(cfg["c"])
    c.h = float(cfg["h"])
    return c


def pps_smc_log_evidence(spec: Mapping, y, lambdas, cfg: Mapping, seed: int, first_run: int = 0,
                         device="cuda", stream=None):
    """log p(y_s | lambda_s) per set s (device FP64 tensor)."""
    import torch
    yy = np.ascontiguousarray(y, np.int32).reshape(-1, len(spec["dose"]))
    lam = np.ascontiguousarray(lambdas, np.float64).reshape(-1, 2)
    n = yy.shape[0]
    assert lam.shape[0] == n
    out = torch.empty(n, dtype=torch.float64, device=device)
    _check(lib().pps_smc_log_evidence(ctypes.byref(make_bioassay(spec)), yy.ctypes.data,
                                      lam.ctypes.data, n, ctypes.byref(make_smc_config(cfg)), seed,
                                      first_run, int(out.data_ptr()), _stream(stream)))
    return out


def pps_wip_test(spec: Mapping, lambdas, n_data: int, cfg: Mapping, seed: int, alpha: float,
                 with_pvalues: bool = True, device="cuda", stream=None) -> dict:
    """Alg. 2 over the rows of `lambdas` (row 0 = the base prior): device
    tensors log_z0, log_zk (and pvalues), host array gamma."""
    import torch
    lam = np.ascontiguousarray(lambdas, np.float64).reshape(-1, 2)
    k = lam.shape[0]
    z0 = torch.empty((k, n_data), dtype=torch.float64, device=device)
    zk = torch.empty((k, n_data), dtype=torch.float64, device=device)
    pv = torch.empty((k, n_data), dtype=torch.float64, device=device) if with_pvalues else None
    gamma = np.zeros(k, np.float64)
    _check(lib().pps_wip_test(ctypes.byref(make_bioassay(spec)), lam.ctypes.data, k, n_data,
                              ctypes.byref(make_smc_config(cfg)), seed, alpha, int(z0.data_ptr()),
                              int(zk.data_ptr()), _ptr(pv), gamma.ctypes.data, _stream(stream)))
    return {"log_z0": z0, "log_zk": zk, "pvalues": pv, "gamma": gamma}


BEGE_NPAR = 11


def pps_bege_loglik(theta, r, n_omega: int = 100, with_logdens: bool = False, device="cuda",
                    stream=None) -> dict:
    """BEGE log-likelihoods (Sec. 4.2) of the rows of `theta` (n x 11) against
    the returns r_0..r_T: device FP64 tensors loglik (n) and, if asked for,
    logdens (n x T).  theta and r may be host arrays or device tensors."""
    import torch
    th = torch.as_tensor(np.asarray(theta, np.float64) if not isinstance(theta, torch.Tensor)
                         else theta, dtype=torch.float64, device=device).reshape(-1, BEGE_NPAR)
    rr = torch.as_tensor(np.asarray(r, np.float64) if not isinstance(r, torch.Tensor) else r,
                         dtype=torch.float64, device=device).reshape(-1)
    th = th.contiguous()
    rr = rr.contiguous()
    n, T = th.shape[0], rr.shape[0] - 1
    ll = torch.empty(n, dtype=torch.float64, device=device)
    ld = torch.empty((n, T), dtype=torch.float64, device=device) if with_logdens else None
    _check(lib().pps_bege_loglik(int(th.data_ptr()), n, int(rr.data_ptr()), T, n_omega,
                                 int(ll.data_ptr()), _ptr(ld), _stream(stream)))
    return {"loglik": ll, "logdens": ld}


def pps_bege_count_ops(theta, r, n_omega: int = 100, device="cuda", stream=None) -> float:
    """FP64 operations of one pps_bege_loglik call on the same batch."""
    import torch
    th = torch.as_tensor(np.asarray(theta, np.float64) if not isinstance(theta, torch.Tensor)
                         else theta, dtype=torch.float64, device=device).reshape(-1, BEGE_NPAR)
    rr = torch.as_tensor(np.asarray(r, np.float64) if not isinstance(r, torch.Tensor) else r,
                         dtype=torch.float64, device=device).reshape(-1)
    th, rr = th.contiguous(), rr.contiguous()
    ops = ctypes.c_double()
    _check(lib().pps_bege_count_ops(int(th.data_ptr()), th.shape[0], int(rr.data_ptr()),
                                    rr.shape[0] - 1, n_omega, ctypes.byref(ops), _stream(stream)))
    return float(ops.value)


def pps_tb_events(model, sampling: pps_sampling, device="cuda", stream=None) -> dict:
    """Tuberculosis runs: per-draw Gillespie event counts (uint64 as int64)
    and status (0 complete, 1 extinct, 2 truncated), device tensors."""
    import torch
    n = int(sampling.n_draws)
    ev = torch.empty(n, dtype=torch.int64, device=device)
    st = torch.empty(n, dtype=torch.int32, device=device)
    _check(lib().pps_tb_events(ctypes.byref(_model_arg(model)), ctypes.byref(sampling),
                               int(ev.data_ptr()), int(st.data_ptr()), _stream(stream)))
    return {"events": ev, "status": st}
