"""Graph replay of the sweep (GPU only): fb_sweep in chunks replayed from a
captured HIP graph gives the same chain, bit for bit, as direct launches.

Each replay reads its per-sweep arguments from device memory written just
before it, so the checks replay one capture many times, with direct sweeps,
state reads and launch-shape changes (which force a new capture) in between,
and compare state, moments and trace with a context that never uses graphs.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import STATE_KEYS, require_gpu, say
from tests.test_oracle_mlp import constant_model

pytestmark = pytest.mark.gpu


def _same(F, a, b, label, seg=0):
    sa, sb = F.fb_get_state(a, seg), F.fb_get_state(b, seg)
    for k in STATE_KEYS:
        assert np.array_equal(sa[k], sb[k]), (label, k)
    ma, mb = F.fb_summaries(a, seg), F.fb_summaries(b, seg)
    for k in ma:
        assert np.array_equal(np.asarray(ma[k]), np.asarray(mb[k])), (label, k)
    assert np.array_equal(F.fb_trace(a, seg)[0], F.fb_trace(b, seg)[0]), label


@pytest.mark.parametrize("precision,shift", [(0, 0), (1, 0), (1, 1)])
def test_graph_replay_matches_direct_launches(precision, shift):
    F = require_gpu()
    ds = datagen.paper_design_16(G=1300, seed=11)
    opts = dict(burnin=30, tune_start=3, precision=precision, jitter=0, thin=1, trace_genes=9, trace_capacity=200,
                update_mask=F.FB_UPDATE_ALL | (F.FB_SHIFT if shift else 0))
    a = F.fb_create(ds.y, ds.X, ds.h, seed=12, options=F.fb_default_options(**opts))
    b = F.fb_create(ds.y, ds.X, ds.h, seed=12, options=F.fb_default_options(**opts))
    F.fb_set_graph(b, 8)
    assert F.fb_get_graph(b) == 8
    steps = [20, 16, 3, 24]        # chunks of 8 with remainders, burn-in crossed at sweep 30
    for i, n in enumerate(steps):
        if i == 2:                 # a new launch shape: the next chunk is captured again
            F.fb_set_launch(a, 2, 0)
            F.fb_set_launch(b, 2, 0)
        say("graph replay: sweeps", n, "precision", precision, "shift", shift)
        F.fb_sweep(a, n)
        F.fb_sweep(b, n)
        _same(F, a, b, f"after call {i}")
    F.fb_destroy(a)
    F.fb_destroy(b)


def test_graph_replay_batched_segments():
    F = require_gpu()
    meta = [(300, 4), (1000, 16), (77, 8), (2500, 4)]
    dss = [datagen.batched_dataset(k + 1, G, N) for k, (G, N) in enumerate(meta)]
    opts = F.fb_default_options(burnin=10, tune_start=2, precision=1, jitter=1, chains=2, thin=2, trace_genes=5,
                                trace_capacity=40)
    spec = [dict(counts=d.y, X=d.X, h=d.h, seed=200 + k) for k, d in enumerate(dss)]
    a = F.fb_create_batch(spec, opts)
    b = F.fb_create_batch(spec, opts)
    F.fb_set_graph(b, 5)
    for n in (15, 10, 7):
        F.fb_sweep(a, n)
        F.fb_sweep(b, n)
        for seg in range(F.fb_num_segments(a)):
            _same(F, a, b, f"segment {seg}", seg)
    F.fb_destroy(a)
    F.fb_destroy(b)


def test_graph_replay_learned_step_with_shift():
    """The learned proposal (network kernel, MH-only gamma/beta kernel, a few
    fallback genes) and the shift step, replayed from a graph."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=900, seed=12)
    L = ds.L
    mu = np.round(np.random.default_rng(21).uniform(-0.3, 0.3, L) * 64) / 64
    m = constant_model(L, mu, np.round(np.full(L, np.log(0.9)) * 64) / 64)
    mask = (np.random.default_rng(22).uniform(size=ds.G) < 0.1).astype(np.int32)
    opts = F.fb_default_options(burnin=10, tune_start=2, precision=1, jitter=0,
                                update_mask=F.FB_UPDATE_ALL | F.FB_SHIFT)
    ctx = []
    for _ in range(2):
        g = F.fb_create(ds.y, ds.X, ds.h, seed=23, options=opts)
        F.fb_sweep(g, 12)
        from tests.test_gpu_mlp import to_gpu_params
        F.fb_proposal_set(g, to_gpu_params(m, L))
        F.fb_fallback(g, 0, mask)
        F.fb_set_beta_update(g, F.FB_BETA_LEARNED)
        ctx.append(g)
    F.fb_set_graph(ctx[1], 4)
    for n in (8, 9, 4):
        F.fb_sweep(ctx[0], n)
        F.fb_sweep(ctx[1], n)
        _same(F, ctx[0], ctx[1], f"learned {n}")
        assert np.array_equal(F.fb_imh_last(ctx[0]), F.fb_imh_last(ctx[1]))
    for g in ctx:
        F.fb_destroy(g)
