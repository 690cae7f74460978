"""Seeded synthetic workloads shared by the GPU library's callers and the oracle.

This module holds input recipes only -- model specifications, prior
hyperparameters, the lambda grid, the serving job mix -- and none of the
method's arithmetic (no random stream, simulator, discrepancy or tally).  Both
sides turn a specification here into their own argument structures.

A specification is a plain dict::

    {"model": "logistic" | "garch11" | "normal_mean" | "toggle_switch",
     "priors": [(family, a, b), ...],   # family: uniform(a,b) | normal(mu,sd)
                                        #   | lognormal(mu,sd) | point(a)
     "constraint": None | "garch_stationary",
     "x0": X0, "t_end": T, "steps": S, "n_obs": n, "noise_sd": sd,
     "n_cells": C}                      # toggle switch only

The workloads follow the paper's structure (prior-predictive sampling for ABC,
Sec. 3; prior-predictive p-values over a hyperparameter family, Sec. 4.1) on
synthetic models of the same shape: the paper's own genetic toggle switch
(Sec. 3.2: 8000 cells, T = 600, 7 uniform priors, 19 quantiles), a stochastic
logistic SDE observed at 20 times, a GARCH(1,1) return series of length 2000,
and a normal-mean model whose prior predictive has a closed form.  The paper's
toggle-switch measurements are not used: observed quantiles come from a
simulation at a fixed theta inside the prior's support.
"""
from __future__ import annotations

import math

import numpy as np

# Seeds: the observed data set is draw 0 of seed 0 at a fixed theta; sampling
# runs use seed 1 so that no sampled draw reuses the observed noise.
OBS_SEED = 0
OBS_DRAW = 0
SAMPLING_SEED = 1

LOGISTIC_THETA_OBS = (1.0, 100.0, 0.2)
GARCH_THETA_OBS = (5e-5, 0.1, 0.85)
# (mu, sigma, gamma, alpha_u, alpha_v, beta_u, beta_v): a point inside the
# toggle-switch prior's support, used to make the synthetic observed data.
TOGGLE_THETA_OBS = (320.0, 0.25, 0.15, 22.0, 12.0, 4.0, 4.5)
# Priors of Sec. 3.2 (after Bonassi et al.), in the order of theta above.
TOGGLE_PRIORS = [("uniform", 250.0, 400.0), ("uniform", 0.05, 0.5), ("uniform", 0.05, 0.35),
                 ("uniform", 0.0, 50.0), ("uniform", 0.0, 50.0), ("uniform", 0.0, 7.0),
                 ("uniform", 0.0, 7.0)]


def logistic_spec(steps: int = 1000, t_end: float = 10.0, n_obs: int = 20, x0: float = 10.0,
                  theta1=("uniform", 0.0, 2.0), theta2=("uniform", 50.0, 150.0),
                  theta3=("uniform", 0.0, 0.5)) -> dict:
    """dX = th1 X (1 - X/th2) dt + th3 X dW on [0, T], X(0) = X0."""
    return {"model": "logistic", "priors": [theta1, theta2, theta3], "constraint": None,
            "x0": x0, "t_end": t_end, "steps": steps, "n_obs": n_obs, "noise_sd": 0.0}


def logistic_point_spec(theta=LOGISTIC_THETA_OBS, **kw) -> dict:
    """The logistic model with every prior a point mass (used to make y_obs)."""
    return logistic_spec(theta1=("point", theta[0], 0.0), theta2=("point", theta[1], 0.0),
                         theta3=("point", theta[2], 0.0), **kw)


def garch_spec(series_len: int = 2000, omega=("uniform", 1e-6, 1e-4), alpha=("uniform", 0.0, 0.3),
               beta=("uniform", 0.5, 0.99), constraint="garch_stationary") -> dict:
    """GARCH(1,1) returns of length L; priors as listed, alpha + beta < 1."""
    return {"model": "garch11", "priors": [omega, alpha, beta], "constraint": constraint,
            "x0": 0.0, "t_end": 0.0, "steps": series_len, "n_obs": 0, "noise_sd": 0.0}


def garch_point_spec(theta=GARCH_THETA_OBS, series_len: int = 2000) -> dict:
    return garch_spec(series_len, ("point", theta[0], 0.0), ("point", theta[1], 0.0),
                      ("point", theta[2], 0.0), constraint=None)


def normal_mean_spec(n_obs: int = 20, noise_sd: float = 1.0, prior_sd: float = 1.0) -> dict:
    """mu ~ N(0, prior_sd^2), y_j = mu + noise_sd z_j, j = 1..n."""
    return {"model": "normal_mean", "priors": [("normal", 0.0, prior_sd)], "constraint": None,
            "x0": 0.0, "t_end": 0.0, "steps": 0, "n_obs": n_obs, "noise_sd": noise_sd}


def toggle_spec(n_cells: int = 8000, steps: int = 599, dt: float = 1.0, n_quantiles: int = 19,
                x0: float = 10.0, priors=None) -> dict:
    """The genetic toggle switch of Sec. 3.2: C cells, S Euler-Maruyama steps
    of size dt (the paper: T = 600 time points, i.e. 599 steps, dt = 1),
    u(0) = v(0) = x0, summaries = n_quantiles equally spaced quantiles."""
    return {"model": "toggle_switch", "priors": list(priors or TOGGLE_PRIORS),
            "constraint": None, "x0": x0, "t_end": steps * dt, "steps": steps,
            "n_obs": n_quantiles, "noise_sd": 0.0, "n_cells": n_cells}


def toggle_point_spec(theta=TOGGLE_THETA_OBS, **kw) -> dict:
    """The toggle switch with every prior a point mass (used to make y_obs)."""
    return toggle_spec(priors=[("point", float(t), 0.0) for t in theta], **kw)


# Weak-informativity test (Sec. 4.1): the logistic dose-response model of
# Eq. bioassay with the design printed in the paper (M = 4 groups of 5
# animals; the dose of group 4 is used as printed), prior N(0, diag(lambda)^2),
# base lambda_0 = (10, 2.5), K hyperparameters lambda_k ~ U([0.1,10] x
# [0.1,20]), N data sets per hyperparameter, and the SMC settings of the paper
# (N_p = 500, c = 0.01, h = 2.38/sqrt(2)).  alpha (the conflict level) is not
# printed in the paper; 0.05 is used.
BIOASSAY = {"n_trials": [5, 5, 5, 5], "dose": [-0.86, -0.3, -0.05, -0.75]}
WIP_LAMBDA0 = (10.0, 2.5)
WIP_ALPHA = 0.05
SMC_CONFIG = {"n_particles": 500, "max_mcmc": 100, "max_steps": 100, "bisect_iters": 50,
              "c": 0.01, "h": 2.38 / math.sqrt(2.0)}
WIP_TEST = {"name": "wip_bioassay_K400_N400_Np500", "n_lambda": 400, "n_data": 400, "seed": 11}


def wip_lambdas(k: int = 400, seed: int = 11) -> np.ndarray:
    """Rows: lambda_0 (the base prior), then k hyperparameters drawn uniformly
    on [0.1, 10] x [0.1, 20] (the paper's benchmark design)."""
    rng = np.random.default_rng(seed)
    lam = np.empty((k + 1, 2))
    lam[0] = WIP_LAMBDA0
    lam[1:, 0] = rng.uniform(0.1, 10.0, size=k)
    lam[1:, 1] = rng.uniform(0.1, 20.0, size=k)
    return lam


# BEGE volatility model (Sec. 4.2).  theta = (p0, sigma_p, rho_p, phi_p+,
# phi_p-, n0, sigma_n, rho_n, phi_n+, phi_n-, mu) with the paper's eleven
# uniform priors.  The observed S&P series (T = 1099 monthly returns) is not
# available; a series of the same length simulated at BEGE_THETA_OBS stands in
# for it (monthly sd about 0.057, mean about 0.01, a -0.44 crash month,
# negative skew).  The likelihood batch is N_p = 1024 parameter vectors, the
# particle count of the paper's sampler, drawn from the prior (the sampler's
# first likelihood evaluation), with the paper's quadrature N_omega = 100.
BEGE_PRIORS = [(1e-4, 0.5), (1e-4, 0.3), (1e-4, 0.99), (1e-4, 0.5), (1e-4, 0.5),
               (1e-4, 1.0), (1e-4, 0.3), (1e-4, 0.99), (-0.2, 0.1), (1e-4, 0.75),
               (-0.9, 0.9)]
BEGE_THETA_OBS = (0.3, 0.02, 0.9, 0.01, 0.03, 0.04, 0.02, 0.85, 0.01, 0.3, 0.008)
BEGE_SERIES = {"name": "bege_T1099", "T": 1099, "seed": 11}
BEGE_BATCH = {"name": "bege_loglik_T1099_Np1024_Nw100", "n_theta": 1024, "n_omega": 100,
              "seed": 7}


def bege_prior_draws(n: int, seed: int = 7) -> np.ndarray:
    """n parameter vectors (rows of 11) drawn from the BEGE priors."""
    rng = np.random.default_rng(seed)
    lo = np.array([b[0] for b in BEGE_PRIORS])
    hi = np.array([b[1] for b in BEGE_PRIORS])
    return lo + (hi - lo) * rng.uniform(size=(n, len(BEGE_PRIORS)))


# Tuberculosis transmission (App. B): a linear birth-death process of cases
# (birth rate alpha, death rate delta per case) with mutation to new genotypes
# (rate tau per case), simulated event by event from one case until the
# population reaches n_stop cases (the stopping size of Tanaka et al.) or dies
# out, at most max_events events; n_sample cases are then drawn without
# replacement (473 isolates in the San Francisco data the paper cites, not
# available here).  Summaries: distinct genotypes / n_sample and gene
# diversity.  Priors: alpha, delta ~ U(0, 5) with alpha > delta (a growing
# epidemic), tau ~ N(0.198, 0.06735) with tau > 0 (Tanaka et al.'s mutation
# rate prior); the paper prints none.
TB_PRIORS = [("uniform", 0.0, 5.0), ("uniform", 0.0, 5.0), ("normal", 0.198, 0.06735)]
TB_THETA_OBS = (1.0, 0.4, 0.2)
TB_PPS = {"name": "tb_gillespie_N16000_K10000_n473", "n": 16000, "n_stop": 10000, "n_sample": 473,
          "max_events": 1 << 20}


def tb_spec(n_stop: int = 10000, n_sample: int = 473, max_events: int = 1 << 20, priors=None,
            x0: float = 1.0) -> dict:
    return {"model": "tb", "priors": list(priors or TB_PRIORS), "constraint": "tb_supercritical",
            "x0": x0, "steps": max_events, "n_obs": n_sample, "n_cells": n_stop}


def tb_point_spec(theta=TB_THETA_OBS, **kw) -> dict:
    """The tuberculosis model with every prior a point mass (used to make
    the synthetic observed summaries)."""
    return tb_spec(priors=[("point", float(t), 0.0) for t in theta], **kw)


def lambda_grid(n: int = 64, lo: float = 0.05, hi: float = 3.0) -> np.ndarray:
    """n log-spaced values from lo to hi (inclusive)."""
    k = np.arange(n, dtype=np.float64)
    return lo * (hi / lo) ** (k / (n - 1))


def pvalue_spec(steps: int = 1000) -> dict:
    """The p-value batch: th1 ~ LogNormal(0, lambda) (lambda is the log-sd),
    the other priors as in the ABC workload."""
    return logistic_spec(steps=steps, theta1=("lognormal", 0.0, 1.0))


# Named configurations (sizes of the paper-shaped workloads).
ABC_SMALL = {"name": "abc_logistic_n1e4", "n": 10_000, "frac": 0.01}
ABC_LARGE = {"name": "abc_logistic_n1e7", "n": 10_000_000, "pilot_n": 100_000, "pilot_frac": 0.001}
PVALUE_BATCH = {"name": "pvalue_logistic_64lambda_n1e6", "n": 1_000_000, "n_lambda": 64}
SERVING_MIX = {"name": "serving_mix_2000jobs_200hz", "n_jobs": 2000, "rate_hz": 200.0, "seed": 3}
GARCH_CHECK = {"name": "garch11_L2000_n1e6", "n": 1_000_000, "series_len": 2000}
TOGGLE_PPS = {"name": "toggle_switch_C8000_T600_n8064", "n": 8064, "n_cells": 8000, "steps": 599}


def serving_jobs(n_jobs: int = 2000, rate_hz: float = 200.0, seed: int = 3,
                 n_lo: float = 1e3, n_hi: float = 1e6, s_lo: float = 200.0, s_hi: float = 5000.0,
                 n_obs: int = 20, n_lambda: int = 64) -> list[dict]:
    """The serving mix: Poisson arrivals, N and steps log-uniform, half ABC
    (closest 1%) and half p-value jobs at a lambda drawn from the grid."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_jobs)
    arrival = np.cumsum(gaps) - gaps[0]
    n_draws = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_jobs)).astype(np.int64)
    steps_raw = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), size=n_jobs))
    steps = np.maximum(n_obs, (np.rint(steps_raw / n_obs) * n_obs).astype(np.int64))
    kind = rng.integers(0, 2, size=n_jobs)
    lam_idx = rng.integers(0, n_lambda, size=n_jobs)
    jobs = []
    for j in range(n_jobs):
        jobs.append({"arrival_s": float(arrival[j]), "n": int(n_draws[j]), "steps": int(steps[j]),
                     "kind": "abc" if kind[j] == 0 else "pvalue", "lambda_index": int(lam_idx[j]),
                     "seed": 1000 + j})
    return jobs
