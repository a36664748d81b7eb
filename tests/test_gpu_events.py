"""Posterior probabilities of contrast events on the GPU (Section 3.2) against
the FP64 oracle (GPU only).

FP64: the integer counts match the oracle's exactly over free-running sweeps
from a shared state (with and without the shift step), in the counting window
the call sets.  FP32: the chain itself differs from the oracle's by rounding,
so the counts of one FP32 sweep from the oracle's state are compared: an event
decision may differ only where the oracle's contrast sits within FP32 rounding
of its bound.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import require_gpu, say
from tests.test_oracle_events import HETEROSIS

pytestmark = pytest.mark.gpu

EVENTS = HETEROSIS + [[([1, 0, 0, 0, 0], 3.0)], [([0, 1, -1, 0, 0], 0.0), ([0, 0, 0, 0, 1], -0.2)]]


@pytest.mark.parametrize("shift", [0, 1])
def test_event_counts_match_oracle_fp64(oracle_lib, shift):
    F = require_gpu()
    ds = datagen.paper_design_16(G=900, seed=14)
    mask = F.FB_UPDATE_ALL | (F.FB_SHIFT if shift else 0)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=15, burnin=12, tune_start=2, update_mask=mask)
    o.sweep(6)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=15,
                    options=F.fb_default_options(burnin=12, tune_start=2, precision=0, jitter=0, update_mask=mask))
    F.fb_set_state(g, o.get_state())
    o.set_contrasts(EVENTS)
    F.fb_set_contrasts(g, EVENTS, ds.L)
    for n in (10, 30):
        o.sweep(n)
        F.fb_sweep(g, n)
        co, no = o.event_counts()
        cg, ng = F.fb_event_counts(g, len(EVENTS))
        say("events: sweeps counted", ng, "mean probabilities", cg.mean(0) / max(ng, 1))
        assert ng == no
        np.testing.assert_array_equal(cg, co)
    p, n = F.fb_event_probs(g, len(EVENTS))
    assert n == 34 and np.all((p >= 0) & (p <= 1))
    F.fb_destroy(g)


def test_event_counts_fp32_one_sweep(oracle_lib):
    F = require_gpu()
    ds = datagen.paper_design_16(G=3000, seed=16)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=17, burnin=5, tune_start=2)
    o.sweep(20)
    st = o.get_state()
    g = F.fb_create(ds.y, ds.X, ds.h, seed=17,
                    options=F.fb_default_options(burnin=5, tune_start=2, precision=1, jitter=0))
    F.fb_set_state(g, st)
    o.set_contrasts(EVENTS)
    F.fb_set_contrasts(g, EVENTS, ds.L)
    o.sweep(1)
    F.fb_sweep(g, 1)
    co, _ = o.event_counts()
    cg, n = F.fb_event_counts(g, len(EVENTS))
    assert n == 1
    beta_o = o.get_state()["beta"]
    bad = np.argwhere(cg != co)
    # a differing decision must come from a draw that differs (a flipped slice
    # decision) or a contrast within FP32 rounding of its bound
    beta_g = F.fb_get_state(g)["beta"]
    for gi, e in bad:
        close = np.allclose(beta_g[gi], beta_o[gi], rtol=1e-4, atol=1e-5)
        if close:
            margins = [abs(np.dot(v, beta_o[gi]) - b) for v, b in EVENTS[e]]
            assert min(margins) < 1e-4, (gi, e, margins)
    assert len(bad) <= 3 * 2e-3 * ds.G * len(EVENTS) + 2
    F.fb_destroy(g)


def test_event_counts_batched_segments_match_single_runs():
    F = require_gpu()
    dss = [datagen.batched_dataset(k + 1, G, 16) for k, G in enumerate((700, 130, 2000))]
    opts = dict(burnin=5, tune_start=2, precision=1, jitter=1, chains=2)
    b = F.fb_create_batch([dict(counts=d.y, X=d.X, h=d.h, seed=300 + k) for k, d in enumerate(dss)],
                          F.fb_default_options(**opts))
    L = dss[0].L
    F.fb_set_contrasts(b, EVENTS, L)
    F.fb_sweep(b, 25)
    for k, d in enumerate(dss):
        s = F.fb_create(d.y, d.X, d.h, seed=300 + k, options=F.fb_default_options(**opts))
        F.fb_set_contrasts(s, EVENTS, L)
        F.fb_sweep(s, 25)
        for ch in range(2):
            cb, nb = F.fb_event_counts(b, len(EVENTS), 2 * k + ch)
            cs, ns = F.fb_event_counts(s, len(EVENTS), ch)
            assert nb == ns == 20
            np.testing.assert_array_equal(cb, cs)
        F.fb_destroy(s)
    F.fb_destroy(b)
