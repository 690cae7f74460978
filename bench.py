#!/usr/bin/env python3
"""Benchmark of the prior-predictive sampler on one MI355X.

Workload (default): ABC rejection on the stochastic logistic SDE,
N = 1e7 prior draws, 1000 Euler-Maruyama steps each, 20 observations,
accepted at the fixed tolerance eps = the 0.1% distance quantile of the FP64
oracle's 1e5-draw pilot (stored in tests/golden/observed.json).  One step =
one ``abc_sample`` call: prior draws, simulation, distances, ordered
compaction of the accepted draws and their FP64 posterior moments, results
copied back to the host.

Prints one JSON line.  ``roofline`` reports the dominant kernel (the
persistent simulation kernel) against the VALU issue peak; its duration is
measured with HIP events that the library records around the kernel on the
caller's stream.  ``cpu_baseline`` times the FP64 oracle on a bounded sample
of the same workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "prior-predictive sims/s + % FP32 VALU peak vs plain GPU; p50/p99 job latency"

# MI355X VALU issue peak: 256 CUs x 128 FP32 lanes per CU per cycle x 2.4 GHz
# = 7.86e13 lane-operations/s, i.e. the published 157.3 TFLOP/s FP32 vector
# peak with an FMA counted as one operation (two flops).
CUS, LANES_PER_CU, CLOCK = 256, 128, 2.4e9
VALU_PEAK_OPS = CUS * LANES_PER_CU * CLOCK  # 7.86e13 lane-ops/s
# Published FP64 vector peak (an FMA counted as two operations).
FP64_PEAK_TFLOPS = 78.6

# Algorithmic VALU lane-operations of the logistic path (see the design notes):
#   Philox4x32-10 call: 10 rounds x (2 widening 32x32->64 multiplies + 4 xor) = 60
#   Box-Muller pair: radius uniform (funnel shift, subtract), log2, scale,
#                    sqrt, angle (funnel shift, and-or, and for two of the
#                    three pairs a shift of word 3), cos, sin, 2 multiplies
#                    = 12   -> 36 per call (6 normals)
#   Euler-Maruyama step: 3 fma + max = 4
#   observation: difference, Kahan (4) for rho^2, Kahan (4) for the sum = 9
#   prior draw: 3 Philox calls + 3 uniform transforms ~ 250 per draw
OPS_PHILOX = 60
OPS_BM_PAIR = 12
NORMALS_PER_CALL = 6
OPS_EM = 4
OPS_OBS = 9
OPS_PRIOR = 250


def ops_per_draw(steps: int, n_obs: int) -> float:
    per_step = (OPS_PHILOX + NORMALS_PER_CALL // 2 * OPS_BM_PAIR) / NORMALS_PER_CALL + OPS_EM
    return steps * per_step + n_obs * OPS_OBS + OPS_PRIOR


# A lambda group (p-value grids): 32 lambda values of one draw per lane share
# the normals; each member adds its EM update and its Kahan mean (4 per
# observation).  The lambda'd parameter's variate is drawn once per draw (one
# Philox call + the FP64 Box-Muller, 72); each member applies its own prior to
# it and forms its EM constants (a + b z, exp, two products / quotients, two
# roundings: 7).
GROUP_LPL = 32
OPS_PRIOR_VARIATES = 72
OPS_PRIOR_MEMBER = 7


def ops_per_group_draw(steps: int, n_obs: int, lpl: int = GROUP_LPL) -> float:
    """Executed lane-operations of one draw of one lambda group."""
    per_step = (OPS_PHILOX + NORMALS_PER_CALL // 2 * OPS_BM_PAIR) / NORMALS_PER_CALL + lpl * OPS_EM
    return (steps * per_step + n_obs * lpl * 4 + OPS_PRIOR + OPS_PRIOR_VARIATES
            + lpl * OPS_PRIOR_MEMBER)


def ops_per_grid_draw_one_normal_set(steps: int, n_obs: int, n_lambda: int) -> float:
    """Lane-operations of one draw under a whole grid with its normals counted
    once (the work the method needs under common random numbers)."""
    return ops_per_group_draw(steps, n_obs, n_lambda)


# GARCH(1,1) step: the normal (16) + sqrt, 2 multiplies, 2 fma for the
# variance, 4 moment sums, b_t, 10 lag products = 36, plus 14 Kahan folds
# (4 ops) every 20 steps = 2.8; closing algebra and prior ~ 600 per draw.
GARCH_OPS_PER_STEP = 38.8
GARCH_OPS_PER_DRAW_FIXED = 600


# Toggle switch (Sec. 3.2), per cell-step: a third of a Philox call (20),
# one Box-Muller pair for (xi_u, xi_v) (12), and per gene the power
# exp2(beta log2 level) (3), the Hill factor 1 / (1 + p) (2), the drift
# and noise updates and the boundary (5) = 52; per cell the measurement
# (power, scale, two adds, boundary: 7), half a pair for eta (6) and a
# linear-time share of the quantile selection (2); per draw the 7 prior
# values (~600).  The LDS bitonic sort that does the selection is not
# counted beyond that linear share.
TSW_OPS_PER_CELL_STEP = 52
TSW_OPS_PER_CELL = 15
TSW_OPS_PER_DRAW = 600


def toggle_ops_per_draw(n_cells: int, steps: int) -> float:
    return n_cells * (steps * TSW_OPS_PER_CELL_STEP + TSW_OPS_PER_CELL) + TSW_OPS_PER_DRAW


# Device sources of each profiled kernel: HBM traffic taken from the PMC
# counters is reported only while these files hash to the digest recorded
# with the counters.
KERNEL_SOURCES = {
    "simulate": ("pps_device.hpp", "pps_internal.hpp", "pps_kernels.hip"),
    "smc": ("pps_device.hpp", "pps_smc.hpp", "pps_smc.hip"),
    "bege": ("pps_bege.hpp", "pps_bege.hip"),
}


def kernel_source_digest(family: str) -> str:
    csrc = os.path.join(ROOT, "paper_1902_09046_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[family]:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(key: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(key)
    if not e or e.get("kernel_source_sha256") != kernel_source_digest(e.get("sources", "simulate")):
        return None
    return e["bytes_per_launch"]


# Published FP32 vector peak (an FMA counted as two flops).
FP32_PEAK_TFLOPS = 157.3


def measured_fp32(key: str, kernel_ms: float):
    """The FP32 FLOP view of a kernel's VALU work from the rocprofv3 counter
    run under profiles/ (64 x (ADD_F32 + MUL_F32 + TRANS_F32 + 2 FMA_F32) per
    dispatch), rated against this run's kernel time, with the instruction
    classes the FLOP counters do not see; null once the sources changed."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or not kernel_ms or kernel_ms <= 0:
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(key)
    if not e or "fp32" not in e or \
            e.get("kernel_source_sha256") != kernel_source_digest(e.get("sources", "simulate")):
        return None
    x = e["fp32"]
    tflops = x["flops_per_launch"] / (kernel_ms * 1e-3) / 1e12
    return {"tflops": round(tflops, 3), "peak": FP32_PEAK_TFLOPS,
            "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
            "weighted_issue_frac": x.get("weighted_issue_frac"),
            "insts_per_launch": x.get("insts")}


def measured_issue(key: str):
    """VALU issue fraction of a kernel from the rocprofv3 counter runs under
    profiles/ (wave64 VALU instructions x 2 SIMD cycles, FP64 arithmetic x 4,
    over the SIMD cycles of the dispatch), while its sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(key)
    if not e or "issue" not in e or \
            e.get("kernel_source_sha256") != kernel_source_digest(e.get("sources", "simulate")):
        return None
    return e["issue"]["frac"]


def time_calls(P, torch, fn, warmup: int, reps: int, warm_s: float = 0.25):
    """Wall time per call (host clock, synchronised) and mean kernel time.
    Warm-up: at least `warmup` calls and at least `warm_s` seconds of them, so
    that the GPU clock has ramped up after the host-only oracle legs."""
    t0 = time.perf_counter()
    k = 0
    while k < warmup or time.perf_counter() - t0 < warm_s:
        fn()
        torch.cuda.synchronize()
        k += 1
    t0 = time.perf_counter()
    ks = []
    for _ in range(reps):
        fn()
        ks.append(P.pps_last_kernel_ms())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, sum(ks) / len(ks)


def serving_bench(P, torch, W, golden, n_jobs: int, rate_hz: float):
    """The serving mix: open-loop Poisson arrivals through the server (latency
    percentiles), then every job submitted at once, batched vs plain."""
    import numpy as np
    jobs_spec = W.serving_jobs(n_jobs=n_jobs, rate_hz=rate_hz, seed=W.SERVING_MIX["seed"])
    ob = golden["logistic_S1000"]
    lam = W.lambda_grid(64)
    jobs = []
    draw_steps = 0
    for js in jobs_spec:
        s = P.make_sampling(js["n"], 0, js["seed"])
        if js["kind"] == "abc":
            jobs.append(P.make_abc_job(W.logistic_spec(steps=js["steps"]), ob["y_obs"], s,
                                       P.PPS_EPS_TOP_FRACTION, 0.01))
        else:
            jobs.append(P.make_pvalue_job(W.pvalue_spec(steps=js["steps"]), 0, P.PPS_LOGNORMAL,
                                          float(lam[js["lambda_index"]]), s, ob["t_obs"]))
        draw_steps += js["n"] * js["steps"]
    need = sum(P.pps_job_arena_bytes(j) for j in jobs)
    arena = torch.empty(need + (64 << 20), dtype=torch.uint8, device="cuda")
    total_draws = sum(js["n"] for js in jobs_spec)
    out = {"jobs": n_jobs, "rate_hz": rate_hz, "draws": total_draws, "sde_steps": draw_steps}

    # open loop: arrivals at their Poisson times; latency = submit -> visible
    print(f"bench: serving open loop {n_jobs} jobs at {rate_hz}/s", file=sys.stderr, flush=True)
    cfg = P.make_server_config(arena, epoch_ms=2.0, max_active=1024)
    with P.Server(cfg) as srv:
        # untimed: 32 jobs at once, so that both epoch slots build the graphs
        # of the forms the mix uses (built on first use)
        for jid in [srv.submit(j) for j in jobs[:32]]:
            while srv.poll(jid)[0] == P.PPS_PENDING:
                time.sleep(0.0005)
            srv.release(jid)
        warm = srv.stats()
        warm_epochs, warm_busy = int(warm.epochs), float(warm.busy_s)
        t0 = time.perf_counter()
        ids = []
        for js, j in zip(jobs_spec, jobs):
            delay = js["arrival_s"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(j))
        lat = []
        for jid in ids:
            while True:
                rc, r = srv.poll(jid)
                if rc != P.PPS_PENDING:
                    break
                time.sleep(0.0005)
            if rc not in (P.PPS_OK, P.PPS_ETRUNC):
                raise RuntimeError(f"serving job failed with status {rc}")
            lat.append(r.t_done - r.t_submit)
        wall = time.perf_counter() - t0
        st = srv.stats()
    lat = np.array(lat)
    out["open_loop"] = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                        "mean_ms": round(float(lat.mean()) * 1e3, 3), "wall_s": round(wall, 3),
                        "epochs": int(st.epochs) - warm_epochs, "gpu_busy_s": round(st.busy_s - warm_busy, 3)}

    # saturated: all jobs at t = 0, continuous batching vs one job per launch;
    # each policy first runs the first 64 jobs untimed (the batch runner's
    # epoch graphs are built on first use of each epoch form)
    sat = {}
    for name, pol in (("batched", P.PPS_POLICY_BATCHED), ("plain", P.PPS_POLICY_PLAIN)):
        P.pps_run_batch(jobs[:64], P.make_server_config(arena, epoch_ms=8.0, max_active=1024,
                                                        policy=pol))
        print(f"bench: serving saturated {name}", file=sys.stderr, flush=True)
        cfg = P.make_server_config(arena, epoch_ms=8.0, max_active=1024, policy=pol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = P.pps_run_batch(jobs, cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bad = [r.status for r in res if r.status not in (P.PPS_OK, P.PPS_ETRUNC)]
        if bad:
            raise RuntimeError(f"saturated {name}: job status {bad[0]}")
        sat[name] = {"wall_s": round(dt, 4), "sims_per_s": round(total_draws / dt, 1),
                     "sde_steps_per_s": round(draw_steps / dt, 1)}
    sat["batched_over_plain"] = round(sat["plain"]["wall_s"] / sat["batched"]["wall_s"], 3)
    out["saturated"] = sat
    return out


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000, help="prior draws per step")
    ap.add_argument("--cpu-sample", type=int, default=8_000_000,
                    help="draws of the oracle's timed sample (0 disables the CPU baseline)")
    ap.add_argument("--only-main", action="store_true",
                    help="skip the p-value batch, GARCH, toggle-switch, weak-informativity and "
                         "serving workloads")
    ap.add_argument("--serving-jobs", type=int, default=2000,
                    help="jobs of the serving mix (0 skips it)")
    ap.add_argument("--launch-shape", default="",
                    help="block,draws_per_lane,unroll of the simulation kernel instead of autotuning "
                         "(profiling runs pin the shape so that every run times the same kernel)")
    ap.add_argument("--cell-block", type=int, default=0,
                    help="workgroup size of the toggle-switch kernel instead of autotuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size (1 GiB read + 1 GiB written), for scaling
    the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": nbytes, "calibrate_copy_bytes_written": nbytes,
                      "copies": 3}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this benchmark runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding of draw ranges is described in the design notes, not built)",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    import numpy as np
    import torch

    import paper_1902_09046_amd as P
    import pps_workloads as W

    torch.cuda.set_device(0)
    with open(os.path.join(ROOT, "tests", "golden", "observed.json")) as f:
        golden = json.load(f)
    y_obs = np.array(golden["logistic_S1000"]["y_obs"])
    eps = golden["abc_n1e7_pilot"]["eps"]
    steps_em, n_obs = 1000, 20
    spec = W.logistic_spec(steps=steps_em, n_obs=n_obs)
    model = P.make_model(spec)
    n = args.n
    sampling = P.make_sampling(n, 0, W.SAMPLING_SEED)
    capacity = max(1024, n // 500)
    idx = torch.empty(capacity, dtype=torch.int64, device="cuda")
    th = torch.empty((3, capacity), dtype=torch.float32, device="cuda")
    dd = torch.empty(capacity, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    P.pps_set_timing(True)
    if args.launch_shape:
        shape = tuple(int(v) for v in args.launch_shape.split(","))
        P.pps_set_launch_shape(0, *shape)
        tune = {"best": shape, "from_cache": False}
        print(f"bench: launch shape {shape} (given)", file=sys.stderr, flush=True)
    else:
        # tuned on the workload's own size: a 2^21-draw probe has ranked a
        # shape first that runs 5 % slower at 1e7 draws
        tune = P.pps_autotune(model, n, use_cache=True)
        print(f"bench: autotuned launch shape {tune['best']} (cache: {tune['from_cache']})",
              file=sys.stderr, flush=True)
    print(f"bench: warmup {args.warmup} x abc_sample N={n}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        P.abc_sample(model, y_obs, sampling, P.PPS_EPS_FIXED, eps, capacity, idx, th, dd)
    kernel_ms, fin_ms = [], []
    stats = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, stats = P.abc_sample(model, y_obs, sampling, P.PPS_EPS_FIXED, eps, capacity, idx, th, dd)
        kernel_ms.append(P.pps_last_kernel_ms())
        fin_ms.append(P.pps_last_finalize_ms())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    print(f"bench: timed {args.steps} steps in {elapsed:.3f}s; accepted {stats['n_accepted']}",
          file=sys.stderr, flush=True)

    value = n * args.steps / elapsed
    k_ms = float(np.mean(kernel_ms))
    ops = ops_per_draw(steps_em, n_obs) * n
    achieved = ops / (k_ms * 1e-3) / 1e12
    peak = VALU_PEAK_OPS / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "TOP/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic("k_simulate_path_abc_n1e7"),
                "valu_issue_frac_counters": measured_issue("k_simulate_path_abc_n1e7"),
                "fp32_flops_counters": measured_fp32("k_simulate_path_abc_n1e7", k_ms),
                "kernel": "k_simulate<block=%d,path,dpl=%d,unroll=%d>" % tuple(tune["best"]),
                "kernel_ms": round(k_ms, 4),
                "ops_per_draw": ops_per_draw(steps_em, n_obs)}

    # The accept step of Alg. 1 on the same 1e7 distances: its HBM rate on
    # algorithmic bytes (rho read once per pass, 4 B per draw; records
    # written, idx 8 B + theta 4 B per parameter + rho 4 B), timed by HIP
    # events around the finalisation inside the call's graph.  Fixed eps:
    # count and write passes.  Closest fraction 0.1 %: three radix-select
    # histogram passes first.
    rec_bytes = 8 + 4 * 3 + 4
    compaction = {}
    fixed_ms = float(np.mean(fin_ms))
    fixed_bytes = 2 * 4 * n + stats["n_accepted"] * rec_bytes
    compaction["fixed_eps"] = {
        "ms": round(fixed_ms, 4), "records": stats["n_accepted"], "passes_over_rho": 2,
        "algorithmic_bytes": fixed_bytes,
        "GB_per_s": round(fixed_bytes / (fixed_ms * 1e-3) / 1e9, 1),
        "traffic": measured_traffic("abc_finalize_fixed_n1e7"),
        "kernels": "k_compact_count, k_compact_scan, k_compact_write, k_moments_final"}
    top_ms = []
    for _ in range(1 + 3):
        _, tstats = P.abc_sample(model, y_obs, sampling, P.PPS_EPS_TOP_FRACTION, 0.001, capacity,
                                 idx, th, dd)
        top_ms.append(P.pps_last_finalize_ms())
    tms = float(np.mean(top_ms[1:]))
    top_bytes = 5 * 4 * n + tstats["n_accepted"] * rec_bytes
    compaction["top_fraction"] = {
        "ms": round(tms, 4), "records": tstats["n_accepted"], "passes_over_rho": 5,
        "algorithmic_bytes": top_bytes,
        "GB_per_s": round(top_bytes / (tms * 1e-3) / 1e9, 1),
        "traffic": measured_traffic("abc_finalize_top_n1e7"),
        "kernels": "k_sel_hist x3, k_sel_pick x3, then the fixed-eps kernels"}
    compaction["note"] = ("rho (40 MB) was just written by the simulation and is re-read "
                          "from the last-level cache, so the rate can exceed HBM's 8 TB/s")

    workloads = {}
    if not args.only_main:
        # Plain ABC rejection at the small size (N = 1e4, closest 1 %, k = 100):
        # the GPU call, and the FP64 oracle on the same draws, timed on the
        # host cores, with the accept sets compared.
        n0 = 10_000
        s0 = P.make_sampling(n0, 0, W.SAMPLING_SEED)
        wall0, _ = time_calls(P, torch, lambda: P.abc_sample(
            model, y_obs, s0, P.PPS_EPS_TOP_FRACTION, 0.01, capacity, idx, th, dd), 2, 5)
        g0 = P.abc(spec, y_obs, W.SAMPLING_SEED, 0, n0, P.PPS_EPS_TOP_FRACTION, 0.01)
        small = {"ms": round(wall0 * 1e3, 4), "sims_per_s": round(n0 / wall0, 1),
                 "accepted": g0["n_accepted"]}
        if args.cpu_sample > 0:
            import oracle
            c0 = time.perf_counter()
            o0 = oracle.abc(spec, y_obs, W.SAMPLING_SEED, 0, n0, oracle.EPS_TOP_FRACTION, 0.01)
            c1 = time.perf_counter()
            sym = set(g0["idx"].cpu().numpy().tolist()) ^ set(o0["idx"].tolist())
            small["oracle"] = {
                "s": round(c1 - c0, 4), "sims_per_s": round(n0 / (c1 - c0), 1),
                "cores": oracle.threads(), "sample": "the whole run (FP64)",
                "accept_set_sym_diff": len(sym),
                "eps_rel_diff": float(f"{abs(g0['eps_used'] - o0['eps_used']) / o0['eps_used']:.3g}")}
        workloads["abc_logistic_n1e4_top1pct"] = small
        # 64-lambda p-value batch, 1e6 draws per lambda, one launch.
        t_obs = golden["logistic_S1000"]["t_obs"]
        pspec = W.pvalue_spec(steps=steps_em)
        lam = W.lambda_grid(64)
        pn = 1_000_000
        print("bench: p-value batch 64 x 1e6", file=sys.stderr, flush=True)
        wall, kms = time_calls(P, torch, lambda: P.prior_pred_pvalue(
            pspec, 0, P.PPS_LOGNORMAL, lam, P.make_sampling(pn, 0, W.SAMPLING_SEED), t_obs), 1, 3)
        pops = ops_per_group_draw(steps_em, n_obs) * pn * (64 // GROUP_LPL)
        pops1 = ops_per_grid_draw_one_normal_set(steps_em, n_obs, 64) * pn
        workloads["pvalue_logistic_64lambda_n1e6"] = {
            "sims_per_s": round(64 * pn / wall, 1), "ms_per_batch": round(wall * 1e3, 3),
            "kernel_ms": round(kms, 3), "valu_frac": round(pops / (kms * 1e-3) / VALU_PEAK_OPS, 4),
            "valu_frac_one_normal_set": round(pops1 / (kms * 1e-3) / VALU_PEAK_OPS, 4),
            "kernel": "k_simulate_group<256,%d>" % GROUP_LPL,
            "traffic": measured_traffic("k_simulate_group_pvalue_64x1e6"),
            "valu_issue_frac_counters": measured_issue("k_simulate_group_pvalue_64x1e6"),
            "fp32_flops_counters": measured_fp32("k_simulate_group_pvalue_64x1e6", kms)}
        if args.cpu_sample > 0:
            # the oracle on the first 1e4 draws of every lambda, timed, and the
            # device's counts on the same draws: equal for lambda <= 1; above,
            # draws in the chaotic regime of the logistic map may flip
            import oracle
            psn = 10_000
            c0 = time.perf_counter()
            po = oracle.pvalue(pspec, 0, "lognormal", lam, W.SAMPLING_SEED, 0, psn, t_obs)
            c1 = time.perf_counter()
            pc, _ = P.prior_pred_pvalue(pspec, 0, P.PPS_LOGNORMAL, lam,
                                        P.make_sampling(psn, 0, W.SAMPLING_SEED), t_obs)
            pdiff = np.abs(np.asarray(pc, np.int64) - po["count_ge"].astype(np.int64))
            small = np.asarray(lam) <= 1.0
            workloads["pvalue_logistic_64lambda_n1e6"]["oracle"] = {
                "sims_per_s": round(64 * psn / (c1 - c0), 1), "cores": oracle.threads(),
                "sample": f"draws [0, {psn}) of each of the 64 lambda values (FP64)",
                "count_diff_lambda_le_1": int(pdiff[small].max()),
                "count_diff_lambda_gt_1_max": int(pdiff[~small].max())}
        # GARCH(1,1) prior-predictive check: 1e6 series of length 2000,
        # 14 summaries per draw written out, then tail-area tallies.
        gspec = W.garch_spec(series_len=2000)
        gn = 1_000_000
        gth = torch.empty((3, gn), dtype=torch.float32, device="cuda")
        gsm = torch.empty((14, gn), dtype=torch.float32, device="cuda")
        print("bench: GARCH 1e6 x 2000", file=sys.stderr, flush=True)
        wall, kms = time_calls(P, torch, lambda: P.pps_simulate(
            gspec, P.make_sampling(gn, 0, W.SAMPLING_SEED), None, gth, gsm, None, None), 1, 3)
        gops = (GARCH_OPS_PER_STEP * 2000 + GARCH_OPS_PER_DRAW_FIXED) * gn
        workloads["garch11_L2000_n1e6_summaries"] = {
            "sims_per_s": round(gn / wall, 1), "ms": round(wall * 1e3, 3), "kernel_ms": round(kms, 3),
            "valu_frac": round(gops / (kms * 1e-3) / VALU_PEAK_OPS, 4),
            "kernel": "k_simulate<256,garch>",
            "traffic": measured_traffic("k_simulate_garch_L2000_n1e6"),
            "valu_issue_frac_counters": measured_issue("k_simulate_garch_L2000_n1e6"),
            "fp32_flops_counters": measured_fp32("k_simulate_garch_L2000_n1e6", kms)}
        if args.cpu_sample > 0:
            # the device's FP32 streaming summaries of the first 1e4 draws
            # against the oracle's FP64 two-pass ones, each error divided by
            # its bar's scale (bar 1e-5): variance and kurtosis relative, the
            # signed mean and skewness relative to the sums over absolute
            # terms, the ten squared-return ACFs absolute
            import oracle
            gsn = 10_000
            c0 = time.perf_counter()
            go = oracle.simulate(gspec, W.SAMPLING_SEED, 0, gsn)["summ"]
            c1 = time.perf_counter()
            gd = gsm[:, :gsn].cpu().numpy().T.astype(np.float64)
            ge = np.abs(gd - go) / oracle.garch_bar_scales(gspec, W.SAMPLING_SEED, range(gsn))
            gerr = {"mean": ge[:, 0], "var": ge[:, 1], "skew": ge[:, 2], "kurt": ge[:, 3],
                    "acf": ge[:, 4:].max(axis=1)}
            workloads["garch11_L2000_n1e6_summaries"]["error_vs_oracle"] = {
                "bar": 1e-5, **{k: {"max": float(f"{v.max():.3g}"),
                                    "median": float(f"{np.median(v):.3g}")}
                                for k, v in gerr.items()}}
            workloads["garch11_L2000_n1e6_summaries"]["oracle"] = {
                "sims_per_s": round(gsn / (c1 - c0), 1), "cores": oracle.threads(),
                "sample": f"draws [0, {gsn}), two-pass FP64 summaries"}
        # The paper's own prior-predictive run (Sec. 3.2, Table A.1): the
        # genetic toggle switch, N = 8064 draws x 8000 cells x 599 steps,
        # each draw reduced to 19 quantiles; ABC keeps the closest 1 %.
        tspec = W.toggle_spec()
        tn, tc, ts = W.TOGGLE_PPS["n"], W.TOGGLE_PPS["n_cells"], W.TOGGLE_PPS["steps"]
        ty = np.array(golden["toggle_C8000_T600"]["y_obs"])
        tcap = 128
        tidx = torch.empty(tcap, dtype=torch.int64, device="cuda")
        tth = torch.empty((7, tcap), dtype=torch.float32, device="cuda")
        tdd = torch.empty(tcap, dtype=torch.float32, device="cuda")
        if args.cell_block:
            P.pps_set_launch_shape(P.CLASS_CELLS, args.cell_block, 1, 1)
            cell_block = args.cell_block
        else:
            cell_block = P.pps_autotune(tspec, 2048, use_cache=True)["best"][0]
        print(f"bench: toggle switch {tn} x {tc} cells x {ts} steps (block {cell_block})",
              file=sys.stderr, flush=True)
        tsamp = P.make_sampling(tn, 0, W.SAMPLING_SEED)
        wall, kms = time_calls(P, torch, lambda: P.abc_sample(
            tspec, ty, tsamp, P.PPS_EPS_TOP_FRACTION, 0.01, tcap, tidx, tth, tdd), 1, 3)
        tops = toggle_ops_per_draw(tc, ts) * tn
        tw = {"sims_per_s": round(tn / wall, 1), "cell_steps_per_s": round(tn * tc * ts / wall, 1),
              "ms": round(wall * 1e3, 3), "kernel_ms": round(kms, 3),
              "valu_frac": round(tops / (kms * 1e-3) / VALU_PEAK_OPS, 4),
              "kernel": f"k_simulate_cells<{cell_block}>",
              "traffic": measured_traffic("k_simulate_cells_toggle_n8064"),
              "valu_issue_frac_counters": measured_issue("k_simulate_cells_toggle_n8064"),
              "fp32_flops_counters": measured_fp32("k_simulate_cells_toggle_n8064", kms),
              "paper_context": {"table": "A.1", "seconds": 69.0, "cpu": "Xeon Gold 6140",
                                "threads": 16, "code": "C, AVX512, FP64",
                                "ratio_to_gpu": round(69.0 / wall, 1)}}
        if args.cpu_sample > 0:
            import oracle
            tns = 32
            c0 = time.perf_counter()
            oracle.simulate(tspec, W.SAMPLING_SEED, 0, tns, y_obs=ty)
            c1 = time.perf_counter()
            tw["oracle"] = {"sims_per_s": round(tns / (c1 - c0), 3), "cores": oracle.threads(),
                            "sample": f"draws [0, {tns}), simulation and summaries (FP64)"}
        workloads["toggle_switch_C8000_T600_n8064"] = tw
        # The weak-informativity test (Sec. 4.1, Table A.2's run): K = 400
        # hyperparameters plus the base, N = 400 data sets each, one adaptive
        # SMC evidence sampler with N_p = 500 particles per data set and prior.
        wlam = W.wip_lambdas(W.WIP_TEST["n_lambda"], seed=W.WIP_TEST["seed"])
        wn = W.WIP_TEST["n_data"]
        print(f"bench: weak-informativity test {wlam.shape[0]} x {wn} (N_p = "
              f"{W.SMC_CONFIG['n_particles']})", file=sys.stderr, flush=True)
        wall, kms = time_calls(P, torch, lambda: P.pps_wip_test(
            W.BIOASSAY, wlam, wn, W.SMC_CONFIG, W.WIP_TEST["seed"], W.WIP_ALPHA), 1, 3)
        runs = 2 * wlam.shape[0] * wn
        ww = {"smc_runs_per_s": round(runs / wall, 1), "ms": round(wall * 1e3, 3),
              "kernel_ms": round(kms, 3), "smc_runs": runs, "kernel": "k_smc<512> (FP64)",
              "traffic": measured_traffic("k_smc_wip_K400_N400"),
              "valu_issue_frac_counters": measured_issue("k_smc_wip_K400_N400"),
              "paper_context": {"table": "A.2", "seconds": 90.0, "cpu": "Xeon Gold 6140",
                                "threads": 16, "code": "C, AVX512, FP64",
                                "ratio_to_gpu": round(90.0 / wall, 1)}}
        if args.cpu_sample > 0:
            import oracle
            sl, sn = wlam[:6], 200
            c0 = time.perf_counter()
            oracle.wip_test(W.BIOASSAY, sl, sn, W.SMC_CONFIG, W.WIP_TEST["seed"], W.WIP_ALPHA)
            c1 = time.perf_counter()
            ww["oracle"] = {"smc_runs_per_s": round(2 * 6 * sn / (c1 - c0), 1),
                            "cores": oracle.threads(),
                            "sample": f"6 priors x {sn} data sets (FP64, the same algorithm)"}
        workloads["wip_bioassay_K400_N400_Np500"] = ww
        # BEGE log-likelihood batch (Sec. 4.2): the N_p = 1024 particles of
        # the paper's sampler, drawn from the prior (its first likelihood
        # evaluation), against a T = 1099 return series, N_omega = 100.
        bb = W.BEGE_BATCH
        bser = np.array(golden["bege_T1099"]["r"])
        bT = len(bser) - 1
        bth = torch.tensor(W.bege_prior_draws(bb["n_theta"], seed=bb["seed"]), device="cuda")
        brd = torch.tensor(bser, device="cuda")
        print(f"bench: BEGE log-likelihood {bb['n_theta']} x T={bT} (N_omega = {bb['n_omega']})",
              file=sys.stderr, flush=True)
        bops = P.pps_bege_count_ops(bth, brd, bb["n_omega"])
        wall, kms = time_calls(P, torch, lambda: P.pps_bege_loglik(bth, brd, bb["n_omega"]), 1, 5)
        bach = bops / (kms * 1e-3) / 1e12
        bw = {"loglik_per_s": round(bb["n_theta"] / wall, 1),
              "densities_per_s": round(bb["n_theta"] * bT / wall, 1),
              "ms": round(wall * 1e3, 3), "kernel_ms": round(kms, 3),
              "kernel": "k_bege_density<64> (FP64)",
              "roofline": {"bound": "alu", "achieved": round(bach, 3), "peak": FP64_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(bach / FP64_PEAK_TFLOPS, 4),
                           "ops_per_launch": bops,
                           "traffic": measured_traffic("k_bege_density_T1099_Np1024")},
                           "valu_issue_frac_counters": measured_issue("k_bege_density_T1099_Np1024"),
              "paper_context": {"table": "A.3", "what": "whole SMC inference (N_p = 1024), "
                                "not one likelihood batch", "seconds": 3115.0,
                                "cpu": "Xeon E5-2680v3", "threads": 16, "code": "C, AVX2, FP64"}}
        if args.cpu_sample > 0:
            import oracle
            bs = 128
            bsample = W.bege_prior_draws(bb["n_theta"], seed=bb["seed"])[:bs]
            c0 = time.perf_counter()
            oracle.bege_loglik_batch(bsample, bser, bb["n_omega"])
            c1 = time.perf_counter()
            bw["oracle"] = {"loglik_per_s": round(bs / (c1 - c0), 2), "cores": oracle.threads(),
                            "sample": f"the first {bs} of the {bb['n_theta']} vectors (FP64, "
                                      "the same quadrature)"}
        workloads[bb["name"]] = bw
        # Tuberculosis prior predictive (App. B, Tables B.1/B.2's largest
        # run: N = 16000 samples): Gillespie runs to a population of 10000
        # cases (cap 2^20 events), 473 cases sampled, ABC keeps the closest
        # 1 %.  One run per 64-lane workgroup, runs from the tile queue.
        tb = W.TB_PPS
        tspec_tb = W.tb_spec(n_stop=tb["n_stop"], n_sample=tb["n_sample"], max_events=tb["max_events"])
        ty_tb = np.array(golden["tb_K10000_n473"]["y_obs"])
        print(f"bench: tuberculosis {tb['n']} runs to {tb['n_stop']} cases", file=sys.stderr, flush=True)
        tsamp_tb = P.make_sampling(tb["n"], 0, W.SAMPLING_SEED)
        tcap_tb = 256
        tidx_tb = torch.empty(tcap_tb, dtype=torch.int64, device="cuda")
        tth_tb = torch.empty((3, tcap_tb), dtype=torch.float32, device="cuda")
        tdd_tb = torch.empty(tcap_tb, dtype=torch.float32, device="cuda")
        ev_tb = P.pps_tb_events(tspec_tb, tsamp_tb)
        events_tb = int(ev_tb["events"].sum().item())
        longest_tb = int(ev_tb["events"].max().item())
        status_tb = np.bincount(ev_tb["status"].cpu().numpy(), minlength=3).tolist()
        wall, kms = time_calls(P, torch, lambda: P.abc_sample(
            tspec_tb, ty_tb, tsamp_tb, P.PPS_EPS_TOP_FRACTION, 0.01, tcap_tb, tidx_tb, tth_tb, tdd_tb), 1, 3)
        tbw = {"sims_per_s": round(tb["n"] / wall, 1), "events_per_s": round(events_tb / wall, 1),
               "ms": round(wall * 1e3, 3), "kernel_ms": round(kms, 3), "events": events_tb,
               "complete_extinct_truncated": status_tb,
               "kernel": "k_simulate_tb<64> (one run per workgroup, counts in LDS)",
               "valu_issue_frac_counters": measured_issue("k_simulate_tb_N16000_K10000"),
               "cycles_per_event_per_workgroup": round(kms * 1e-3 * CLOCK * 4 * CUS / events_tb, 1),
               # a run is a serial chain: the batch cannot end before its
               # longest run, so the latency view is the kernel time per
               # event of that run (an upper bound on one event's latency)
               "longest_run_events": longest_tb,
               "cycles_per_event_longest_run": round(kms * 1e-3 * CLOCK / max(longest_tb, 1), 1),
               "paper_context": {"table": "B.2", "seconds": 183.0, "cpu": "Xeon Gold 6140",
                                 "threads": 4, "code": "C, AVX512",
                                 "note": "the paper's runs stop and sample by rules it does not print"}}
        if args.cpu_sample > 0:
            import oracle
            tbs = 256
            c0 = time.perf_counter()
            oo = oracle.tb_simulate(tspec_tb, W.SAMPLING_SEED, 0, tbs)
            c1 = time.perf_counter()
            tbw["oracle"] = {"sims_per_s": round(tbs / (c1 - c0), 2),
                             "events_per_s": round(float(oo["events"].sum()) / (c1 - c0), 1),
                             "cores": oracle.threads(),
                             "sample": f"draws [0, {tbs}) (the same runs, linear genotype lookup)"}
        workloads[tb["name"]] = tbw
        if args.serving_jobs > 0:
            workloads["serving_mix"] = serving_bench(P, torch, W, golden, args.serving_jobs,
                                                     W.SERVING_MIX["rate_hz"])

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        ns = min(args.cpu_sample, n)
        print(f"bench: cpu_baseline oracle on {ns} draws", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        oracle.abc(spec, y_obs, W.SAMPLING_SEED, 0, ns, oracle.EPS_FIXED, eps, capacity=0)
        c1 = time.perf_counter()
        cpu = {"value": round(ns / (c1 - c0), 1), "unit": "sims/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"draws [0, {ns}) of the same workload (FP64, OpenMP static partition)"}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "sims/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "abc_logistic_sde_n1e7_S1000_fixed_eps", "n_draws": n,
                   "em_steps": steps_em, "n_obs": n_obs, "eps": eps,
                   "accepted": stats["n_accepted"], "launch_shape": list(tune["best"])},
        "sde_steps_per_s": round(value * steps_em, 1),
        "roofline": roofline,
        "compaction": compaction,
        "cpu_baseline": cpu,
        "workloads": workloads,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
