"""Two lanes per gene in the beta draws of the slice sweep (GPU only).

fb_set_beta_lanes(c, 2) draws each beta_gl with a pair of lanes: the two
step-out directions at once, shrink candidates two at a time.  Points,
decisions and counters are those of the one-lane draw, so:

* one lane and two lanes give the same chain bit for bit (state, per-draw
  records, moments, trace, event counts; FP64 and FP32; batches of datasets
  with different L, the L <= 8 kernels; graph replay);
* with two lanes the FP64 chain matches the oracle draw for draw, edge cases
  and the shrink cap included.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import STATE_KEYS, require_gpu, say
from tests.test_gpu_parity import _compare_fp64, _edge_datasets, _make_pair

pytestmark = pytest.mark.gpu


def _same(F, a, b, label, seg=0, events=0):
    sa, sb = F.fb_get_state(a, seg), F.fb_get_state(b, seg)
    for k in STATE_KEYS:
        assert np.array_equal(sa[k], sb[k]), (label, k)
    ma, mb = F.fb_summaries(a, seg), F.fb_summaries(b, seg)
    for k in ma:
        assert np.array_equal(np.asarray(ma[k]), np.asarray(mb[k])), (label, k)
    da, db = F.fb_debug_counts(a, seg), F.fb_debug_counts(b, seg)
    for k in ("eps", "gam", "beta", "hyp"):
        assert np.array_equal(da[k], db[k]), (label, k)
    assert np.array_equal(F.fb_trace(a, seg)[0], F.fb_trace(b, seg)[0]), label
    if events:
        assert np.array_equal(F.fb_event_counts(a, events, seg)[0], F.fb_event_counts(b, events, seg)[0]), label


@pytest.mark.parametrize("precision,shift", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_two_lanes_give_the_one_lane_chain(precision, shift):
    """Also with the shift step, which then runs inside the pair kernel."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=1500, seed=41)
    opts = F.fb_default_options(burnin=15, tune_start=3, precision=precision, jitter=0, debug_counts=1, thin=1,
                                trace_genes=11, trace_capacity=80,
                                update_mask=F.FB_UPDATE_ALL | (F.FB_SHIFT if shift else 0))
    a = F.fb_create(ds.y, ds.X, ds.h, seed=42, options=opts)
    b = F.fb_create(ds.y, ds.X, ds.h, seed=42, options=opts)
    F.fb_set_beta_lanes(b, 2)
    assert F.fb_get_beta_lanes(b) == 2 and F.fb_get_beta_lanes(a) == 1
    ev = [[(np.array([0.0, 2.0, 0.0, 1.0, 0.0]), 0.0)], [(np.array([0.0, 0.0, 1.0, 0.0, 0.0]), -0.1)]]
    for g in (a, b):
        F.fb_set_contrasts(g, ev, 5)
    for i, n in enumerate((10, 9, 25)):
        if i == 2:
            F.fb_set_graph(a, 6)
            F.fb_set_graph(b, 6)
        say("one vs two beta lanes: sweeps", n, "precision", precision, "shift", shift)
        F.fb_sweep(a, n)
        F.fb_sweep(b, n)
        _same(F, a, b, f"call {i}", events=2)
    F.fb_destroy(a)
    F.fb_destroy(b)


@pytest.mark.parametrize("precision", [0, 1])
def test_two_lanes_batched_segments(precision):
    """Datasets with L = 2, 3, 5 and one with L = 7 (the L <= 8 kernel), two
    chains each, in one context."""
    F = require_gpu()
    meta = [(300, 4), (1000, 16), (77, 8)]
    dss = [datagen.batched_dataset(k + 1, G, N) for k, (G, N) in enumerate(meta)]
    H2 = np.array([[1.0, 1.0], [1.0, -1.0]])
    H8 = np.kron(np.kron(H2, H2), H2)[:, :7]
    dss.append(datagen.simulate(130, H8, [3.0] + [0.0] * 6, [1.5] + [0.3] * 6, seed=43))
    opts = F.fb_default_options(burnin=8, tune_start=2, precision=precision, jitter=1, chains=2, debug_counts=1)
    spec = [dict(counts=d.y, X=d.X, h=d.h, seed=50 + k) for k, d in enumerate(dss)]
    a = F.fb_create_batch(spec, opts)
    b = F.fb_create_batch(spec, opts)
    F.fb_set_beta_lanes(b, 2)
    for n in (6, 11):
        F.fb_sweep(a, n)
        F.fb_sweep(b, n)
        for seg in range(F.fb_num_segments(a)):
            _same(F, a, b, f"segment {seg}", seg)
    F.fb_destroy(a)
    F.fb_destroy(b)


def test_two_lanes_fp64_parity_100_sweeps(oracle_lib):
    ds = datagen.small_two_group(G=1000, seed=0)
    F, g, o = _make_pair(oracle_lib, ds, seed=44, burnin=40, tune_start=5, precision=0)
    F.fb_set_beta_lanes(g, 2)
    F.fb_set_state(g, o.get_state())
    for it in range(100):
        assert o.sweep(1) == 0
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"two lanes sweep {it + 1}")
    F.fb_destroy(g)


_EDGES = [e for e in _edge_datasets() if e[0] in ("G1", "G65_ragged", "N1_L1", "K0", "K3_w0small", "L7_N8",
                                                   "huge_counts", "paper_N16")]


@pytest.mark.parametrize("name,ds,kw", _EDGES, ids=[e[0] for e in _EDGES])
def test_two_lanes_fp64_parity_edge_cases(oracle_lib, name, ds, kw):
    say("two lanes edge case", name, ds.y.shape)
    F, g, o = _make_pair(oracle_lib, ds, seed=3, burnin=10, tune_start=2, precision=0, **dict(kw))
    F.fb_set_beta_lanes(g, 2)
    F.fb_set_state(g, o.get_state())
    for it in range(20):
        o.sweep(1)
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"{name} sweep {it + 1}")
    F.fb_destroy(g)


def test_two_lanes_fp64_parity_with_shift_step(oracle_lib):
    ds = datagen.paper_design_16(G=700, seed=47)
    F, g, o = _make_pair(oracle_lib, ds, seed=48, burnin=20, tune_start=3, precision=0,
                         update_mask=0xFE | (1 << 11))
    F.fb_set_beta_lanes(g, 2)
    F.fb_set_state(g, o.get_state())
    for it in range(30):
        assert o.sweep(1) == 0
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"two lanes with shift, sweep {it + 1}")
    F.fb_destroy(g)


def test_two_lanes_shrink_cap_matches(oracle_lib):
    """A cap of 2 shrink candidates and a huge window: capped draws keep x0
    and raise FB_ENUMERIC, with the counters of the oracle."""
    ds = datagen.small_two_group(G=200, seed=1)
    F, g, o = _make_pair(oracle_lib, ds, seed=5, burnin=0, tune_start=0, precision=0, cap=2, w0=30.0)
    F.fb_set_beta_lanes(g, 2)
    F.fb_set_state(g, o.get_state())
    assert o.sweep(1) == -4
    F.fb_sweep(g, 1)
    with pytest.raises(F.FbError) as e:
        F.fb_sync(g)
    assert e.value.code == F.FB_ENUMERIC
    _compare_fp64(F, g, o, "two lanes, shrink cap")
    F.fb_destroy(g)


def test_autotune_with_beta_lanes_leaves_the_chain_unchanged():
    F = require_gpu()
    ds = datagen.paper_design_16(G=2000, seed=45)
    opts = F.fb_default_options(burnin=20, tune_start=2, precision=1, jitter=0)
    a = F.fb_create(ds.y, ds.X, ds.h, seed=46, options=opts)
    b = F.fb_create(ds.y, ds.X, ds.h, seed=46, options=opts)
    for g in (a, b):
        F.fb_sweep(g, 12)
    spw, fuse, ms, tried = F.fb_autotune(b, 5)
    say("autotune: spw", spw, "fuse", fuse, "lanes", F.fb_get_beta_lanes(b), "ms", ms)
    for g in (a, b):
        F.fb_sweep(g, 15)
    sa, sb = F.fb_get_state(a), F.fb_get_state(b)
    for k in STATE_KEYS:
        assert np.array_equal(sa[k], sb[k]), k
    F.fb_destroy(a)
    F.fb_destroy(b)
