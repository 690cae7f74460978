"""Pins of the oracle's per-summary tail-area tally (Sec. 4.1, the tail-area
form of Eq. pppv applied to each summary): count_s = #{i : S_s(D_i) >= obs_s},
the comparison inclusive.

The tally is checked against a count made here in numpy over the per-draw
summaries the oracle's simulator returns, for the three summary-vector models
(GARCH(1,1), the toggle switch of Sec. 3.2, the tuberculosis model of App. B).
Each observed vector is built so that every summary index matters and the tie
case is exercised: one simulated draw's own summaries (every comparison of that
draw is an equality), the per-summary medians (a shifted summary index moves
the counts), and values just above and below a simulated value."""
import numpy as np
import pytest

import oracle
import pps_workloads as W

SEED = 5


def _specs():
    return {
        "garch": (W.garch_spec(series_len=200), 300),
        "toggle": (W.toggle_spec(n_cells=200, steps=40, n_quantiles=7), 96),
        "tb": (W.tb_spec(n_stop=120, n_sample=40, max_events=20000), 200),
    }


def _numpy_count(summ, obs):
    return (summ >= np.asarray(obs)[None, :]).sum(axis=0).astype(np.uint64)


@pytest.mark.parametrize("name", ["garch", "toggle", "tb"])
def test_summary_tally_equals_count_over_simulated_summaries(name):
    spec, n = _specs()[name]
    sim = oracle.simulate(spec, SEED, 0, n)
    summ = sim["summ"]
    ns = summ.shape[1]
    assert ns == oracle.n_summaries(spec) and ns >= 2
    med = np.median(summ, axis=0)
    # the observed vectors: a simulated draw itself (ties on every summary),
    # the medians, and each summary of a draw nudged one ulp up and down
    j = n // 3
    cases = [summ[j].copy(), med, np.nextafter(summ[j], np.inf), np.nextafter(summ[j], -np.inf),
             np.full(ns, -np.inf), np.full(ns, np.inf)]
    for obs in cases:
        got = oracle.summary_tally(spec, SEED, 0, n, obs)
        assert np.array_equal(got, _numpy_count(summ, obs)), (name, obs, got)
    # the tie case: draw j's own summaries count it on every summary, and one
    # ulp above them it drops out of each count whose summary is not shared
    tie = oracle.summary_tally(spec, SEED, 0, n, summ[j])
    above = oracle.summary_tally(spec, SEED, 0, n, np.nextafter(summ[j], np.inf))
    dup = (summ == summ[j][None, :]).sum(axis=0)
    assert np.array_equal(tie - above, dup.astype(np.uint64))
    # the summary index matters: counts against the medians are near n/2 per
    # summary, while a vector of one summary's median repeated is not the same
    # tally unless the summaries coincide
    assert oracle.summary_tally(spec, SEED, 0, n, np.full(ns, np.inf)).sum() == 0
    assert np.all(oracle.summary_tally(spec, SEED, 0, n, np.full(ns, -np.inf)) == n)


def test_summary_tally_draw_range():
    """A tally over [first, first + n) is the sum of tallies over a split."""
    spec, n = _specs()["garch"]
    obs = np.median(oracle.simulate(spec, SEED, 0, n)["summ"], axis=0)
    whole = oracle.summary_tally(spec, SEED, 0, n, obs)
    a = oracle.summary_tally(spec, SEED, 0, 117, obs)
    b = oracle.summary_tally(spec, SEED, 117, n - 117, obs)
    assert np.array_equal(whole, a + b)
    sim = oracle.simulate(spec, SEED, 117, n - 117)
    assert np.array_equal(b, _numpy_count(sim["summ"], obs))
