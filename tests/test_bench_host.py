"""Host-side contract of bench.py (no GPU): the one-GPU refusal, the operation
counts behind the roofline figures, and the rule that measured HBM traffic is
reported only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused_with_a_message(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                       capture_output=True, text=True, env={**os.environ, **env}, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_operation_counts_of_the_roofline():
    # per EM step: a sixth of a Philox call (60), a Box-Muller pair per two
    # normals (3 x 12 per call of six normals), the EM update (4)
    assert bench.ops_per_draw(1000, 20) == 1000 * ((60 + 36) / 6 + 4) + 20 * 9 + 250 == 20430
    # a draw-group of 32 lambda values: one normal per step, 32 EM updates,
    # 32 Kahan means per observation, the shared theta, the lambda'd
    # parameter's variate once, 32 member transforms
    assert bench.ops_per_group_draw(1000, 20) == 1000 * (16 + 128) + 20 * 128 + 250 + 72 + 32 * 7 == 147106
    # the 64-lambda grid with its normals counted once per draw
    assert bench.ops_per_grid_draw_one_normal_set(1000, 20, 64) == 1000 * (16 + 256) + 20 * 256 + 250 + 72 + 64 * 7
    # toggle switch: 52 per cell-step, 15 per cell, 600 per draw
    assert bench.toggle_ops_per_draw(8000, 599) == 8000 * (599 * 52 + 15) + 600
    assert bench.VALU_PEAK_OPS == 256 * 128 * 2.4e9


def test_kernel_source_families_exist():
    csrc = os.path.join(ROOT, "paper_1902_09046_amd", "csrc")
    for fam, names in bench.KERNEL_SOURCES.items():
        for n in names:
            assert os.path.exists(os.path.join(csrc, n)), (fam, n)
        assert len(bench.kernel_source_digest(fam)) == 64


def test_traffic_is_reported_only_for_the_measured_sources(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    entries = {k: e for k, e in table.items() if isinstance(e, dict) and "bytes_per_launch" in e}
    assert entries
    for key, e in entries.items():
        # the recorded digest: the measured bytes
        monkeypatch.setattr(bench, "kernel_source_digest", lambda fam, d=e["kernel_source_sha256"]: d)
        assert bench.measured_traffic(key) == e["bytes_per_launch"]
        # any other source text: nothing
        monkeypatch.setattr(bench, "kernel_source_digest", lambda fam: "0" * 64)
        assert bench.measured_traffic(key) is None
        # the bytes are the scaled counters of the entry
        assert e["bytes_per_launch"] == round((e["fetch_kib"] * e["fetch_scale"] +
                                               e["write_kib"] * e["write_scale"]) * 1024)
    assert bench.measured_traffic("no such kernel") is None


def test_fp32_counter_view_follows_the_measured_sources(monkeypatch):
    """The FP32 FLOP view (64 x (ADD + MUL + TRANS + 2 FMA) wave instructions
    per dispatch) is rated against the run's own kernel time and reported
    only for the sources it was measured on."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    entries = {k: e for k, e in table.items() if isinstance(e, dict) and "fp32" in e}
    assert "k_simulate_path_abc_n1e7" in entries
    for key, e in entries.items():
        x = e["fp32"]
        # the flops are the counters' FP32 arithmetic classes, FMA twice
        assert x["flops_per_launch"] >= 64 * x["insts"]["f32_add_mul_fma"]
        assert x["insts"]["valu"] >= x["insts"]["f32_add_mul_fma"] + x["insts"]["trans_f32"]
        monkeypatch.setattr(bench, "kernel_source_digest", lambda fam, d=e["kernel_source_sha256"]: d)
        v = bench.measured_fp32(key, 2.0)
        assert v["tflops"] == pytest.approx(x["flops_per_launch"] / 2e-3 / 1e12, rel=1e-3, abs=1e-3)
        assert v["frac"] == pytest.approx(v["tflops"] / 157.3, abs=1e-4)
        assert bench.measured_fp32(key, 4.0)["tflops"] == pytest.approx(v["tflops"] / 2, rel=1e-3, abs=1e-3)
        monkeypatch.setattr(bench, "kernel_source_digest", lambda fam: "0" * 64)
        assert bench.measured_fp32(key, 2.0) is None
    assert bench.measured_fp32("no such kernel", 1.0) is None
