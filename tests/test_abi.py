"""The C ABI without a GPU: libpps.so loads, exports every function that
include/pps.h declares, its structs have the layout the binding assumes, and
argument validation answers before any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pps.h")


@pytest.fixture(scope="module")
def P():
    import paper_1902_09046_amd as P
    from paper_1902_09046_amd import build
    if not os.path.exists(P.LIB_PATH):
        build.build()
    return P


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("abc_sample", "prior_pred_pvalue", "pps_simulate", "pps_philox", "pps_normals",
              "pps_summary_tally", "pps_strerror", "pps_last_error", "pps_n_summaries"):
        assert n in names


def test_library_exports_every_declared_symbol(P):
    L = P.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(ln.split()[-1] for ln in out.splitlines() if " T " in ln)
    assert set(declared_functions()) <= exported
    # no bare poll/submit that would interpose libc
    assert "poll" not in exported and "submit" not in exported


_LAYOUT_PROG = r"""
#include <stdio.h>
#include <stddef.h>
#include "pps.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(pps_prior), sizeof(pps_model), sizeof(pps_sampling), sizeof(pps_abc_stats));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", offsetof(pps_model, prior), offsetof(pps_model, constraint),
         offsetof(pps_model, x0), offsetof(pps_model, t_end), offsetof(pps_model, steps),
         offsetof(pps_model, n_obs), offsetof(pps_model, noise_sd), offsetof(pps_model, n_cells));
  printf("%zu %zu %zu\n", offsetof(pps_abc_stats, eps_used), offsetof(pps_abc_stats, mean), offsetof(pps_abc_stats, var));
  printf("%zu %zu %zu %zu\n", sizeof(pps_job), sizeof(pps_job_result), sizeof(pps_server_config), sizeof(pps_server_stats));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", offsetof(pps_job, model), offsetof(pps_job, sampling), offsetof(pps_job, y_obs),
         offsetof(pps_job, eps_mode), offsetof(pps_job, capacity), offsetof(pps_job, lambda_param), offsetof(pps_job, lambda), offsetof(pps_job, t_obs));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(pps_job_result, abc), offsetof(pps_job_result, count_ge), offsetof(pps_job_result, acc_idx),
         offsetof(pps_job_result, n_records), offsetof(pps_job_result, record_stride), offsetof(pps_job_result, t_done));
  printf("%zu %zu %zu %zu\n", offsetof(pps_server_config, max_active), offsetof(pps_server_config, epoch_ms), offsetof(pps_server_config, policy),
         offsetof(pps_server_config, stream));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(pps_bioassay), offsetof(pps_bioassay, dose), sizeof(pps_smc_config),
         offsetof(pps_smc_config, bisect_iters), offsetof(pps_smc_config, c), offsetof(pps_smc_config, h));
  return 0;
}
"""


def test_struct_layout_matches_binding(P):
    from paper_1902_09046_amd import _pps as B
    d = tempfile.mkdtemp(prefix="pps_layout_")
    src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
    with open(src, "w") as f:
        f.write(_LAYOUT_PROG)
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    assert sizes == [ctypes.sizeof(B.pps_prior), ctypes.sizeof(B.pps_model),
                     ctypes.sizeof(B.pps_sampling), ctypes.sizeof(B.pps_abc_stats)]
    offs = [int(v) for v in lines[1].split()]
    assert offs == [getattr(B.pps_model, f).offset for f in
                    ("prior", "constraint", "x0", "t_end", "steps", "n_obs", "noise_sd", "n_cells")]
    offs2 = [int(v) for v in lines[2].split()]
    assert offs2 == [getattr(B.pps_abc_stats, f).offset for f in ("eps_used", "mean", "var")]
    assert [int(v) for v in lines[3].split()] == [ctypes.sizeof(B.pps_job), ctypes.sizeof(B.pps_job_result),
                                                  ctypes.sizeof(B.pps_server_config),
                                                  ctypes.sizeof(B.pps_server_stats)]
    assert [int(v) for v in lines[4].split()] == [getattr(B.pps_job, f).offset for f in (
        "model", "sampling", "y_obs", "eps_mode", "capacity", "lambda_param", "lambda_", "t_obs")]
    assert [int(v) for v in lines[5].split()] == [getattr(B.pps_job_result, f).offset for f in (
        "abc", "count_ge", "acc_idx", "n_records", "record_stride", "t_done")]
    assert [int(v) for v in lines[6].split()] == [getattr(B.pps_server_config, f).offset for f in (
        "max_active", "epoch_ms", "policy", "stream")]
    assert [int(v) for v in lines[7].split()] == [
        ctypes.sizeof(B.pps_bioassay), B.pps_bioassay.dose.offset, ctypes.sizeof(B.pps_smc_config),
        B.pps_smc_config.bisect_iters.offset, B.pps_smc_config.c.offset, B.pps_smc_config.h.offset]


def test_wip_validation_without_device(P):
    import pps_workloads as W
    L = P.lib()
    b = P.make_bioassay(W.BIOASSAY)
    cfg = P.make_smc_config(W.SMC_CONFIG)
    lam = np.array([[10.0, 2.5], [1.0, 1.0]])
    g = np.zeros(2)

    def call(b_, cfg_, lam_, n_lambda, n_data, alpha):
        return L.pps_wip_test(ctypes.byref(b_), lam_.ctypes.data, n_lambda, n_data, ctypes.byref(cfg_),
                              1, alpha, 1, 1, None, g.ctypes.data, None)
    for field, bad in [("n_particles", 1), ("n_particles", 1025), ("max_mcmc", 0), ("max_mcmc", 257),
                       ("bisect_iters", 0), ("max_steps", 0)]:
        c2 = P.make_smc_config(W.SMC_CONFIG)
        setattr(c2, field, bad)
        assert call(b, c2, lam, 2, 10, 0.05) == P.PPS_EINVAL
    for field, bad in [("c", 0.0), ("c", 1.0), ("h", 0.0), ("h", float("inf"))]:
        c2 = P.make_smc_config(W.SMC_CONFIG)
        setattr(c2, field, bad)
        assert call(b, c2, lam, 2, 10, 0.05) == P.PPS_EINVAL
    b2 = P.make_bioassay(W.BIOASSAY)
    b2.n_groups = 9
    assert call(b2, cfg, lam, 2, 10, 0.05) == P.PPS_EINVAL
    b3 = P.make_bioassay(W.BIOASSAY)
    b3.n_trials[1] = -1
    assert call(b3, cfg, lam, 2, 10, 0.05) == P.PPS_EINVAL
    assert call(b, cfg, lam, 0, 10, 0.05) == P.PPS_EINVAL
    assert call(b, cfg, lam, 2, 0, 0.05) == P.PPS_EINVAL
    assert call(b, cfg, lam, 2, 10, 0.0) == P.PPS_EINVAL
    assert call(b, cfg, np.array([[10.0, 2.5], [1.0, -1.0]]), 2, 10, 0.05) == P.PPS_EINVAL
    assert L.pps_last_error()
    y_bad = np.array([[6, 0, 0, 0]], np.int32)
    assert L.pps_smc_log_evidence(ctypes.byref(b), y_bad.ctypes.data, lam.ctypes.data, 1, ctypes.byref(cfg),
                                  1, 0, 1, None) == P.PPS_EINVAL


def test_validation_without_device(P):
    import pps_workloads as W
    L = P.lib()
    assert P.pps_n_summaries(W.logistic_spec()) == 20
    assert P.pps_n_summaries(W.garch_spec()) == 14
    assert P.pps_n_summaries(W.normal_mean_spec(n_obs=7)) == 7
    assert P.pps_n_summaries(W.toggle_spec()) == 19
    assert P.pps_n_summaries(W.toggle_spec(n_cells=P.PPS_TSW_MAX_CELLS, n_quantiles=64, steps=1)) == 64
    tsw_six = W.toggle_spec()
    tsw_six["priors"] = tsw_six["priors"][:6]
    tsw_constrained = W.toggle_spec()
    tsw_constrained["constraint"] = "garch_stationary"
    bad = [W.logistic_spec(steps=999), W.logistic_spec(n_obs=0), W.logistic_spec(n_obs=65, steps=65),
           W.garch_spec(series_len=1990), W.logistic_spec(theta1=("uniform", 2.0, 1.0)),
           W.logistic_spec(theta1=("normal", 0.0, -1.0)), W.logistic_spec(t_end=-1.0),
           W.toggle_spec(n_cells=0), W.toggle_spec(n_cells=P.PPS_TSW_MAX_CELLS + 1),
           W.toggle_spec(n_quantiles=0), W.toggle_spec(n_quantiles=65), W.toggle_spec(steps=0),
           W.toggle_spec(dt=-1.0), tsw_six, tsw_constrained]
    for spec in bad:
        assert L.pps_n_summaries(ctypes.byref(P.make_model(spec))) == P.PPS_EINVAL
        assert L.pps_last_error()
    m = P.make_model(W.logistic_spec())
    bad_family = P.make_model(W.logistic_spec())
    bad_family.prior[0].family = 9
    assert L.pps_n_summaries(ctypes.byref(bad_family)) == P.PPS_EINVAL
    st = P._pps.pps_abc_stats()
    y = np.zeros(20)
    s0 = P.make_sampling(0, 0, 1)
    s1 = P.make_sampling(100, 0, 1)
    # N = 0
    assert L.abc_sample(ctypes.byref(m), y.ctypes.data, ctypes.byref(s0), 1, 0.01, 0, None, None, None,
                        ctypes.byref(st), None) == P.PPS_EINVAL
    # NULL y_obs, NULL stats, bad mode, bad fraction, missing buffers with capacity
    assert L.abc_sample(ctypes.byref(m), None, ctypes.byref(s1), 1, 0.01, 0, None, None, None,
                        ctypes.byref(st), None) == P.PPS_EINVAL
    assert L.abc_sample(ctypes.byref(m), y.ctypes.data, ctypes.byref(s1), 1, 0.01, 0, None, None, None,
                        None, None) == P.PPS_EINVAL
    assert L.abc_sample(ctypes.byref(m), y.ctypes.data, ctypes.byref(s1), 7, 0.01, 0, None, None, None,
                        ctypes.byref(st), None) == P.PPS_EINVAL
    assert L.abc_sample(ctypes.byref(m), y.ctypes.data, ctypes.byref(s1), 1, 0.0, 0, None, None, None,
                        ctypes.byref(st), None) == P.PPS_EINVAL
    assert L.abc_sample(ctypes.byref(m), y.ctypes.data, ctypes.byref(s1), 1, 0.01, 5, None, None, None,
                        ctypes.byref(st), None) == P.PPS_EINVAL
    y_bad = y.copy()
    y_bad[3] = np.nan
    assert L.abc_sample(ctypes.byref(m), y_bad.ctypes.data, ctypes.byref(s1), 1, 0.01, 0, None, None,
                        None, ctypes.byref(st), None) == P.PPS_EINVAL
    lam = np.array([1.0, 2.0])
    cnt = np.zeros(2, np.uint64)
    pv = np.zeros(2)
    assert L.prior_pred_pvalue(ctypes.byref(m), 3, 2, lam.ctypes.data, 2, ctypes.byref(s1), 1.0,
                               cnt.ctypes.data, pv.ctypes.data, None) == P.PPS_EINVAL
    assert L.prior_pred_pvalue(ctypes.byref(m), 0, 2, lam.ctypes.data, 0, ctypes.byref(s1), 1.0,
                               cnt.ctypes.data, pv.ctypes.data, None) == P.PPS_EINVAL
    lam_bad = np.array([-1.0, 2.0])  # negative log-sd
    assert L.prior_pred_pvalue(ctypes.byref(m), 0, 2, lam_bad.ctypes.data, 2, ctypes.byref(s1), 1.0,
                               cnt.ctypes.data, pv.ctypes.data, None) == P.PPS_EINVAL
    g = P.make_model(W.garch_spec())
    assert L.prior_pred_pvalue(ctypes.byref(g), 0, 2, lam.ctypes.data, 2, ctypes.byref(s1), 1.0,
                               cnt.ctypes.data, pv.ctypes.data, None) == P.PPS_EINVAL
    assert L.pps_summary_tally(ctypes.byref(m), ctypes.byref(s1), y.ctypes.data, cnt.ctypes.data,
                               None) == P.PPS_EINVAL
    assert L.pps_philox(1, 0, 0, 0, 0, None, None) == P.PPS_EINVAL
    assert L.pps_normals(1, 0, 10, 0, None, None) == P.PPS_EINVAL


def test_job_arena_bytes_and_server_validation(P):
    """Arena sizing and argument checks that answer without a device."""
    import pps_workloads as W
    L = P.lib()
    spec = W.logistic_spec()
    s = P.make_sampling(100_000, 0, 1)
    j = P.make_abc_job(spec, np.zeros(20), s, P.PPS_EPS_TOP_FRACTION, 0.01)
    need = P.pps_job_arena_bytes(j)
    assert need >= 100_000 * 4 + 1000 * (8 + 16 + 4)  # distances + 1000 records
    pj = P.make_pvalue_job(W.pvalue_spec(), 0, P.PPS_LOGNORMAL, 0.5, s, 70.0)
    assert P.pps_job_arena_bytes(pj) == 256
    bad = P.make_pvalue_job(W.pvalue_spec(), 5, P.PPS_LOGNORMAL, 0.5, s, 70.0)
    assert L.pps_job_arena_bytes(ctypes.byref(bad)) == P.PPS_EINVAL
    bad2 = P.make_abc_job(spec, np.zeros(20), s, P.PPS_EPS_TOP_FRACTION, 2.0)
    assert L.pps_job_arena_bytes(ctypes.byref(bad2)) == P.PPS_EINVAL
    cfg = P._pps.pps_server_config()
    h = ctypes.c_void_p()
    assert L.pps_server_create(ctypes.byref(cfg), ctypes.byref(h)) == P.PPS_EINVAL  # no arena
    cfg.arena, cfg.arena_bytes, cfg.max_active, cfg.epoch_ms = 4096, 1 << 20, 0, 1.0
    assert L.pps_server_create(ctypes.byref(cfg), ctypes.byref(h)) == P.PPS_EINVAL  # max_active
    cfg.max_active, cfg.epoch_ms = 8, 0.0
    assert L.pps_server_create(ctypes.byref(cfg), ctypes.byref(h)) == P.PPS_EINVAL  # epoch_ms
    cfg.epoch_ms, cfg.arena = 1.0, 4097
    assert L.pps_server_create(ctypes.byref(cfg), ctypes.byref(h)) == P.PPS_EINVAL  # alignment
    cfg.arena = 4096
    res = (P._pps.pps_job_result * 1)()
    arr = (P._pps.pps_job * 1)(bad)
    assert L.pps_run_batch(arr, 1, ctypes.byref(cfg), res) == P.PPS_EINVAL  # invalid job
    assert L.pps_submit(None, ctypes.byref(j), ctypes.byref(ctypes.c_uint64())) == P.PPS_EINVAL


def test_strerror(P):
    L = P.lib()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, 42):
        assert L.pps_strerror(code)
    assert L.pps_strerror(-6) == b"output truncated to capacity"


def test_bege_validation_without_device(P):
    L = P.lib()
    dev = 1  # never dereferenced: every call below fails validation first

    def call(n_theta, T, n_omega, theta=dev, r=dev, ll=dev):
        return L.pps_bege_loglik(theta, n_theta, r, T, n_omega, ll, None, None)
    for args in [(0, 10, 100), (-1, 10, 100), ((1 << 20) + 1, 10, 100), (4, 0, 100),
                 (4, (1 << 20) + 1, 100), (1 << 20, 1 << 12, 100), (4, 10, 1), (4, 10, 65537)]:
        assert call(*args) == P.PPS_EINVAL, args
    assert call(4, 10, 100, theta=None) == P.PPS_EINVAL
    assert call(4, 10, 100, r=None) == P.PPS_EINVAL
    assert call(4, 10, 100, ll=None) == P.PPS_EINVAL
    assert b"n_omega" in L.pps_last_error() or L.pps_last_error()


def test_bege_count_ops_validation_without_device(P):
    import ctypes as C
    L = P.lib()
    ops = C.c_double()
    assert L.pps_bege_count_ops(1, 4, 1, 10, 100, None, None) == P.PPS_EINVAL
    assert L.pps_bege_count_ops(1, 0, 1, 10, 100, C.byref(ops), None) == P.PPS_EINVAL
    assert L.pps_bege_count_ops(None, 4, 1, 10, 100, C.byref(ops), None) == P.PPS_EINVAL


def test_tb_validation_without_device(P):
    import pps_workloads as W
    assert P.pps_n_summaries(W.tb_spec()) == 2
    bad = [W.tb_spec(n_stop=1), W.tb_spec(n_stop=P.PPS_TB_MAX_POP + 1), W.tb_spec(n_sample=0),
           W.tb_spec(n_sample=P.PPS_TB_MAX_SAMPLE + 1), W.tb_spec(max_events=0), W.tb_spec(x0=0.0),
           W.tb_spec(x0=2.5), W.tb_spec(n_stop=100, x0=101.0)]
    two = W.tb_spec()
    two["priors"] = two["priors"][:2]
    garch_c = W.tb_spec()
    garch_c["constraint"] = "garch_stationary"
    bad += [two, garch_c]
    for spec in bad:
        with pytest.raises(P.PPSError):
            P.pps_n_summaries(spec)
    logistic_tb = W.logistic_spec()
    logistic_tb["constraint"] = "tb_supercritical"
    with pytest.raises(P.PPSError):
        P.pps_n_summaries(logistic_tb)
    L = P.lib()
    m = P.make_model(W.logistic_spec())
    s = P.make_sampling(10, 0, 1)
    import ctypes as C
    assert L.pps_tb_events(C.byref(m), C.byref(s), None, None, None) == P.PPS_EINVAL
