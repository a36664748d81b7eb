"""Pins of the oracle's posterior probabilities of contrast events (CPU only).

Section 3.2 estimates P(v_1^T beta_g > b_1 and ... and v_K^T beta_g > b_K | y)
by the mean, over post-burn-in sweeps, of the indicator of the event at each
sweep.  The oracle keeps integer counts per (gene, event); the pins recount
the indicators from the end-of-sweep states stored sweep by sweep, check the
counting window (after burn-in and after the call), and the events whose
answer is known (always, never, an event and its complement).
"""
import numpy as np

from paper_1606_06659_amd import datagen
from tests.test_golden import heterosis_events

# the paper's high- and low-parent heterosis events for the design of Section 5
# (coefficients 2, 3, 4 in the paper's 1-based numbering are l = 1, 2, 3 here)
HETEROSIS = heterosis_events()      # Section 5 (tests/golden/heterosis_events.txt)


def _recount(states, events, L):
    c = np.zeros((states[0].shape[0], len(events)), np.int64)
    for beta in states:
        for e, ev in enumerate(events):
            ok = np.ones(beta.shape[0], bool)
            for v, b in ev:
                ok &= beta @ np.asarray(v, float) > b
            c[:, e] += ok
    return c


def test_event_counts_match_a_recount(oracle_lib):
    ds = datagen.paper_design_16(G=40, seed=2)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=3, burnin=12, tune_start=2,
                          update_mask=oracle_lib.UPDATE_ALL | (1 << 11))
    o.sweep(5)
    events = HETEROSIS + [[([1, 0, 0, 0, 0], 3.0)], [([0, 1, -1, 0, 0], 0.0), ([0, 0, 0, 0, 1], -0.2)]]
    o.set_contrasts(events)          # at m = 5: counting starts after burn-in, m = 13
    states = []
    for _ in range(40):
        o.sweep(1)
        if o.get_state()["m"] > 12:
            states.append(o.get_state()["beta"].copy())
    counts, n = o.event_counts()
    assert n == len(states) == 33
    np.testing.assert_array_equal(counts, _recount(states, events, ds.L))
    assert counts.min() >= 0 and counts.max() <= n and 0 < counts.sum() < counts.size * n


def test_event_counting_starts_after_the_call(oracle_lib):
    ds = datagen.small_two_group(G=25, seed=4)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=5, burnin=3, tune_start=1)
    o.sweep(10)
    events = [[([0, 1], 0.0)]]
    o.set_contrasts(events)          # after burn-in: only the following sweeps count
    states = []
    for _ in range(15):
        o.sweep(1)
        states.append(o.get_state()["beta"].copy())
    counts, n = o.event_counts()
    assert n == 15
    np.testing.assert_array_equal(counts, _recount(states, events, ds.L))


def test_events_with_known_answers(oracle_lib):
    ds = datagen.small_two_group(G=30, seed=6)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=7, burnin=0, tune_start=0)
    v = np.array([0.3, -1.0])
    events = [[([0.0, 0.0], -1.0)],           # 0 > -1: always
              [([0.0, 0.0], 0.0)],            # 0 > 0: never
              [(v, 0.1)], [(-v, -0.1)],       # an event and its complement (ties have probability 0)
              [(v, 0.1), ([0.0, 0.0], -1.0)]]  # conjunction with an always-true row
    o.set_contrasts(events)
    o.sweep(50)
    counts, n = o.event_counts()
    assert n == 50
    assert np.all(counts[:, 0] == n) and np.all(counts[:, 1] == 0)
    np.testing.assert_array_equal(counts[:, 2] + counts[:, 3], n)
    np.testing.assert_array_equal(counts[:, 4], counts[:, 2])
    assert 0 < counts[:, 2].sum() < 30 * n
