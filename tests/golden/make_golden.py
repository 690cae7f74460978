"""Write the observed data sets used by the tests and the benchmark.

Calls only the FP64 oracle.  The observed data of each workload is one
prior-predictive simulation at a fixed theta (point priors), seed 0, draw 0:

* logistic SDE, theta = (1, 100, 0.2), X0 = 10, T = 10, S = 1000, observed at
  steps 50, 100, ..., 1000 -> ``y_obs`` (20 values) and ``t_obs`` = their mean;
* GARCH(1,1), theta = (5e-5, 0.1, 0.85), L = 2000 -> the 14 summaries;
* genetic toggle switch, theta = (320, 0.25, 0.15, 22, 12, 4, 4.5), C = 8000
  cells, 599 Euler-Maruyama steps of dt = 1 (T = 600 time points), x0 = 10
  -> the 19 quantile summaries ``y_obs`` and ``t_obs`` = their mean (the
  paper's measured cells are not available; this stands in for them);
* BEGE volatility model, theta = (0.3, 0.02, 0.9, 0.01, 0.03, 0.04, 0.02,
  0.85, 0.01, 0.3, 0.008), T = 1099, seed 11 -> the returns r_0..r_T (the
  S&P series of the paper is not available; this stands in for it);
* tuberculosis transmission, theta = (1, 0.4, 0.2), population stop 10000,
  473 cases sampled: the first draw (seed 0) whose epidemic reaches the stop
  size -> (distinct genotypes / 473, gene diversity) (the San Francisco data
  the paper cites are not available; this stands in for them);
* the fixed tolerance of the 1e7-draw ABC workload: the 0.1% distance
  quantile of the oracle's pilot on draws [0, 1e5) of the sampling seed
  (the 100th smallest distance, type-1 inverse empirical CDF).

Values are written with 17 significant digits so they round-trip exactly.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pps_workloads as W  # noqa: E402


def main():
    out = {}
    for steps in (1000,):
        spec = W.logistic_point_spec(steps=steps)
        sim = oracle.simulate(spec, W.OBS_SEED, W.OBS_DRAW, 1)
        y = sim["summ"][0]
        out[f"logistic_S{steps}"] = {
            "theta": list(W.LOGISTIC_THETA_OBS), "seed": W.OBS_SEED, "draw": W.OBS_DRAW,
            "y_obs": [float(repr_) for repr_ in y], "t_obs": float(sim["stat"][0]),
        }
    spec = W.logistic_spec(steps=1000)
    y = out["logistic_S1000"]["y_obs"]
    pilot_n = W.ABC_LARGE["pilot_n"]
    pilot = oracle.abc(spec, y, W.SAMPLING_SEED, 0, pilot_n, oracle.EPS_TOP_FRACTION,
                       W.ABC_LARGE["pilot_frac"], capacity=0)
    out["abc_n1e7_pilot"] = {"seed": W.SAMPLING_SEED, "first": 0, "n": pilot_n,
                             "k": oracle.top_count(W.ABC_LARGE["pilot_frac"], pilot_n),
                             "eps": pilot["eps_used"], "mean": list(pilot["mean"]),
                             "var": list(pilot["var"])}
    gspec = W.garch_point_spec()
    gs = oracle.simulate(gspec, W.OBS_SEED, W.OBS_DRAW, 1)
    out["garch_L2000"] = {"theta": list(W.GARCH_THETA_OBS), "seed": W.OBS_SEED,
                          "draw": W.OBS_DRAW, "summaries": [float(v) for v in gs["summ"][0]]}
    tspec = W.toggle_point_spec()
    ts = oracle.simulate(tspec, W.OBS_SEED, W.OBS_DRAW, 1)
    out["toggle_C8000_T600"] = {"theta": list(W.TOGGLE_THETA_OBS), "seed": W.OBS_SEED,
                                "draw": W.OBS_DRAW, "n_cells": tspec["n_cells"],
                                "steps": tspec["steps"],
                                "y_obs": [float(v) for v in ts["summ"][0]],
                                "t_obs": float(ts["stat"][0])}
    tspec_tb = W.tb_point_spec()
    tb_draw = 0
    while True:
        tr = oracle.tb_simulate(tspec_tb, W.OBS_SEED, tb_draw, 1)
        if tr["status"][0] == oracle.TB_COMPLETE:
            break
        tb_draw += 1
    out["tb_K10000_n473"] = {"theta": list(W.TB_THETA_OBS), "seed": W.OBS_SEED, "draw": tb_draw,
                             "n_stop": tspec_tb["n_cells"], "n_sample": tspec_tb["n_obs"],
                             "events": int(tr["events"][0]),
                             "y_obs": [float(v) for v in tr["summ"][0]]}
    bs = W.BEGE_SERIES
    r = oracle.bege_simulate(W.BEGE_THETA_OBS, bs["T"], bs["seed"])
    out["bege_T1099"] = {"theta": list(W.BEGE_THETA_OBS), "seed": bs["seed"], "T": bs["T"],
                         "r": [float(v) for v in r]}
    path = os.path.join(HERE, "observed.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
