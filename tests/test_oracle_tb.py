"""Pins of the oracle's tuberculosis transmission model (App. B: a linear
birth-death process of cases with mutation to new genotypes, simulated by the
Gillespie direct method; summaries: distinct genotypes and gene diversity of
a sample) against facts fixed outside its code:

* the genotype lookup is numpy's inverse of the cumulative weights, and new
  genotypes go to the lowest empty slot;
* the total number of cases is a random walk stepping up with probability
  alpha/(alpha + delta) at each birth or death, mutations leaving it alone:
  the extinction probability before reaching K cases is the gambler's-ruin
  value, the mean number of events the gambler's-ruin duration divided by the
  probability 1 - tau/(alpha + delta + tau) that an event moves the walk, and
  with delta = 0 every run reaches K after K - 1 births;
* event types occur with the rate fractions (binomial counts over many
  events);
* the summaries of a population taken whole are numpy's distinct count and
  1 - sum (X_i/N)^2; taken by a sample without replacement they average to
  the multivariate hypergeometric expectations;
* the constrained prior keeps alpha > delta and tau > 0 with the right
  conditional law.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import pps_workloads as W


def test_select_is_the_inverse_cumulative_lookup():
    rng = np.random.default_rng(0)
    for _ in range(200):
        x = rng.integers(0, 5, size=int(rng.integers(1, 60))).astype(np.uint32)
        x[rng.random(len(x)) < 0.3] = 0
        if x.sum() == 0:
            x[-1] = 1
        for m in range(int(x.sum())):
            assert oracle.tb_select(x, m) == int(np.searchsorted(np.cumsum(x), m, side="right"))


def test_lowest_empty_slot():
    rng = np.random.default_rng(1)
    for _ in range(200):
        x = rng.integers(0, 3, size=40).astype(np.uint32)
        expect = int(np.argmax(x == 0)) if (x == 0).any() else -1
        assert oracle.tb_lowest_empty(x) == expect


def gamblers_ruin(p, k):
    """P(hit 0 before k from 1) and E[steps] for a walk up w.p. p."""
    q = 1.0 - p
    r = q / p
    ruin = (r - r ** k) / (1.0 - r ** k)
    steps = 1.0 / (q - p) - (k / (q - p)) * (1.0 - r) / (1.0 - r ** k)
    return ruin, steps


@pytest.mark.parametrize("theta,k", [((1.0, 0.8, 0.3), 40), ((2.0, 1.0, 0.5), 60), ((0.7, 0.6, 0.05), 25)])
def test_extinction_and_duration_follow_gamblers_ruin(theta, k):
    runs = [oracle.tb_run(theta, k, 11, d) for d in range(3000)]
    ext = np.array([r["status"] == oracle.TB_EXTINCT for r in runs])
    ev = np.array([r["events"] for r in runs], np.float64)
    for r in runs:
        assert r["status"] in (oracle.TB_EXTINCT, oracle.TB_COMPLETE)
        assert r["n"] == (0 if r["status"] == oracle.TB_EXTINCT else k)
        assert int(r["counts"].sum()) == r["n"]
    a, d, t = theta
    ruin, steps = gamblers_ruin(a / (a + d), k)
    se = math.sqrt(ruin * (1 - ruin) / len(runs))
    assert abs(ext.mean() - ruin) < 4.5 * se, (ext.mean(), ruin)
    mean_events = steps / (1.0 - t / (a + d + t))
    assert abs(ev.mean() / mean_events - 1.0) < 4.5 * ev.std() / math.sqrt(len(runs)) / mean_events


def test_pure_birth_reaches_k_after_k_minus_one_births():
    k = 300
    a, t = 1.3, 0.4
    ev = []
    for d in range(400):
        r = oracle.tb_run((a, 0.0, t), k, 5, d)
        assert r["status"] == oracle.TB_COMPLETE and r["n"] == k
        ev.append(r["events"] - (k - 1))       # the mutations
    ev = np.array(ev, np.float64)
    # mutations between births: negative binomial, mean (k-1) t/a
    mean = (k - 1) * t / a
    var = (k - 1) * (t / a) * (1 + t / a)
    assert abs(ev.mean() - mean) < 4.5 * math.sqrt(var / len(ev))


def test_event_types_follow_the_rates():
    theta = (1.0, 0.9, 0.6)
    tb, td = oracle.tb_thresholds(theta)
    r = theta[0] + theta[1] + theta[2]
    # the thresholds are floor(2^32 alpha/R), floor(2^32 (alpha + delta)/R)
    assert tb == math.floor(theta[0] / r * 2 ** 32) and td == math.floor((theta[0] + theta[1]) / r * 2 ** 32)
    # and the type words of the event stream fall between them in the rate
    # fractions (words 1 and 3 of each block)
    words = np.array([oracle.stream_block(4, 9, b, oracle.TB_PURPOSE_EVENT) for b in range(20000)],
                     np.uint64)
    wt = np.concatenate([words[:, 1], words[:, 3]])
    frac = np.array([(wt < tb).mean(), ((wt >= tb) & (wt < td)).mean(), (wt >= td).mean()])
    expect = np.array(theta) / r
    assert np.all(np.abs(frac - expect) < 4.5 * np.sqrt(expect * (1 - expect) / len(wt)))


def test_whole_population_summaries():
    for d in range(30):
        run = oracle.tb_run((1.2, 0.3, 0.4), 200, 3, d)
        if run["n"] == 0:
            continue
        x = run["counts"].astype(np.int64)
        n = int(x.sum())
        s = oracle.tb_summaries(run["counts"], n + 5, 3, d)   # n_sample > N: all cases
        assert s[0] == (x > 0).sum() / n
        assert s[1] == pytest.approx(1.0 - ((x / n) ** 2).sum(), abs=1e-15)
    assert list(oracle.tb_summaries(np.zeros(10, np.uint32), 5, 1, 1)) == [0.0, 0.0]


def test_sample_summaries_match_hypergeometric_expectations():
    x = np.array([40, 1, 0, 7, 3, 0, 22, 1, 1, 5, 12, 8], np.uint32)
    N, n = int(x.sum()), 30
    g, h = [], []
    for d in range(4000):
        s = oracle.tb_summaries(x, n, 21, d)
        g.append(s[0] * n)
        h.append(s[1])
    g, h = np.array(g), np.array(h)
    eg = sum(1.0 - stats.hypergeom(N, int(xi), n).pmf(0) for xi in x if xi > 0)
    mean = n * x / N
    var = n * (x / N) * (1 - x / N) * (N - n) / (N - 1)
    eh = 1.0 - (var + mean ** 2).sum() / n ** 2
    assert abs(g.mean() - eg) < 4.5 * g.std() / math.sqrt(len(g))
    assert abs(h.mean() - eh) < 4.5 * h.std() / math.sqrt(len(h))
    assert np.all(g <= (x > 0).sum())


def test_prior_constraint():
    spec = W.tb_spec(n_stop=50, n_sample=20)
    o = oracle.tb_simulate(spec, 2, 0, 4000)
    th = o["theta"]
    assert np.all(th[:, 0] > th[:, 1]) and np.all(th[:, 2] > 0)
    # given alpha > delta with both U(0, 5): P(alpha <= a) = (a/5)^2
    assert stats.kstest(th[:, 0], lambda a: np.clip(a / 5.0, 0, 1) ** 2).pvalue > 1e-3
    # tau ~ N(0.198, 0.06735) (truncation at 0 is 3 sd away)
    assert abs(th[:, 2].mean() - 0.198) < 4.5 * 0.06735 / math.sqrt(len(th))


def test_simulate_agrees_with_the_tb_entry_and_caps_events():
    spec = W.tb_spec(n_stop=400, n_sample=50, max_events=3000)
    a = oracle.tb_simulate(spec, 7, 100, 200)
    b = oracle.simulate(spec, 7, 100, 200)
    np.testing.assert_array_equal(a["theta"], b["theta"])
    np.testing.assert_array_equal(a["summ"], b["summ"])
    trunc = a["status"] == oracle.TB_TRUNCATED
    assert np.all(a["events"][trunc] == 3000) and np.all(a["events"] <= 3000)
    assert trunc.any()


def test_observed_summaries_are_the_golden_ones():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "observed.json")) as f:
        g = json.load(f)["tb_K10000_n473"]
    spec = W.tb_point_spec(tuple(g["theta"]), n_stop=g["n_stop"], n_sample=g["n_sample"])
    o = oracle.tb_simulate(spec, g["seed"], g["draw"], 1)
    assert o["status"][0] == oracle.TB_COMPLETE and int(o["events"][0]) == g["events"]
    np.testing.assert_array_equal(o["summ"][0], g["y_obs"])
