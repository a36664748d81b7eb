"""Three-level form (Section 2.3) on the GPU against the oracle (GPU only).

The datasets of a batched context are the groups k; a top level (b, psi)
per chain ties their tau and theta priors.  FP64: free-running sweeps from a
shared state, every draw of every group within a relative 1e-5 with identical
per-draw records, and b, psi and their running moments equal to the
oracle's (the same Philox words, the same sums in the same order); with two
chains, with the exact conjugate draws and the shift step; graph replay
equals direct launches; FP32 keeps the top-level draws of the first sweep
from a shared state.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import STATE_KEYS, require_gpu, say

pytestmark = pytest.mark.gpu

EXACT = 1 << 12
SHIFT = 1 << 11
META = [(300, 11), (77, 12), (1000, 13)]     # (G, data seed) of the groups
TOP = dict(a_b=3.0, b_b=2.0, c0=[1.5, 0.7], seed=77)


def _datasets():
    return [datagen.small_two_group(G=G, seed=s) for G, s in META]


def _pair(oracle_lib, *, precision=0, chains=1, mask=0xFE, burnin=10, top_mask=3):
    F = require_gpu()
    dss = _datasets()
    opts = F.fb_default_options(burnin=burnin, tune_start=2, precision=precision, debug_counts=1, jitter=0,
                                chains=chains, update_mask=mask)
    g = F.fb_create_batch([dict(counts=d.y, X=d.X, h=d.h, seed=500 + k) for k, d in enumerate(dss)], opts)
    F.fb_set_top_level(g, TOP["a_b"], TOP["b_b"], np.array(TOP["c0"]), TOP["seed"], top_mask)
    tops = []
    for ch in range(chains):
        groups = [oracle_lib.Oracle(d.y, d.X, d.h, seed=500 + k, chain=ch, burnin=burnin, tune_start=2,
                                    update_mask=mask) for k, d in enumerate(dss)]
        top = oracle_lib.ThreeLevel(groups, a_b=TOP["a_b"], b_b=TOP["b_b"], c0=np.array(TOP["c0"]),
                                    seed=TOP["seed"], chain=ch, burnin=burnin, top_mask=top_mask)
        for k, o in enumerate(groups):
            F.fb_set_state(g, o.get_state(), k * chains + ch)
        F.fb_set_top(g, ch, top.b, top.psi)
        tops.append(top)
    return F, g, tops


def _compare(F, g, tops, label, chains):
    for ch, top in enumerate(tops):
        t = F.fb_get_top(g, ch)
        np.testing.assert_allclose(t["b"], top.b, rtol=1e-9, err_msg=label)
        np.testing.assert_allclose(t["psi"], top.psi, rtol=1e-9, atol=1e-12, err_msg=label)
        for k, o in enumerate(top.groups):
            seg = k * chains + ch
            so, sg = o.get_state(), F.fb_get_state(g, seg)
            for key in STATE_KEYS:
                err = np.abs(sg[key] - so[key])
                bad = np.argwhere(~(err <= 1e-5 * np.abs(so[key]) + 1e-10))
                assert bad.size == 0, (label, ch, k, key, bad[:5])
            co, cg = o.counts(), F.fb_debug_counts(g, seg)
            for key in ("eps", "gam", "beta", "hyp"):
                assert np.array_equal(co[key], cg[key]), (label, ch, k, key)


@pytest.mark.parametrize("chains,mask", [(1, 0xFE), (2, 0xFE), (1, 0xFE | EXACT | SHIFT)],
                         ids=["one_chain", "two_chains", "exact_shift"])
def test_fp64_three_level_parity(oracle_lib, chains, mask):
    F, g, tops = _pair(oracle_lib, chains=chains, mask=mask)
    for it in range(30):
        say("three-level sweep", it + 1, "chains", chains, "mask", hex(mask))
        for top in tops:
            assert top.sweep(1) == 0
        F.fb_sweep(g, 1)
        _compare(F, g, tops, f"sweep {it + 1}", chains)
    for ch, top in enumerate(tops):
        t = F.fb_get_top(g, ch)
        assert top.count == 20
        np.testing.assert_allclose(t["mean"], top.mean, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(t["msq"], top.msq, rtol=1e-9, atol=1e-12)
        assert t["tries"] == top.tries >= 1
    F.fb_destroy(g)


@pytest.mark.parametrize("top_mask", [1, 2])
def test_fp64_three_level_partial_top(oracle_lib, top_mask):
    """Only b (mask 1) or only psi (mask 2) drawn; the other stays fixed."""
    F, g, tops = _pair(oracle_lib, top_mask=top_mask)
    for it in range(10):
        tops[0].sweep(1)
        F.fb_sweep(g, 1)
        _compare(F, g, tops, f"partial {top_mask} sweep {it + 1}", 1)
    t = F.fb_get_top(g, 0)
    if top_mask == 1:
        assert np.all(t["psi"] == 0.0)
    else:
        assert t["b"] == 1.0
    F.fb_destroy(g)


def test_three_level_graph_replay_matches_direct(oracle_lib):
    """Graph replay with the hyperparameter step on one workgroup per segment
    equals direct launches with one workgroup per chain of draws."""
    F, a, _ = _pair(oracle_lib, chains=2)
    _, b, _ = _pair(oracle_lib, chains=2)
    F.fb_set_graph(b, 6)
    F.fb_set_hyper_split(b, 0)
    for n in (12, 7, 13):
        F.fb_sweep(a, n)
        F.fb_sweep(b, n)
        for ch in range(2):
            ta, tb = F.fb_get_top(a, ch), F.fb_get_top(b, ch)
            assert ta["b"] == tb["b"] and np.array_equal(ta["psi"], tb["psi"])
            assert np.array_equal(ta["mean"], tb["mean"])
        for seg in range(F.fb_num_segments(a)):
            sa, sb = F.fb_get_state(a, seg), F.fb_get_state(b, seg)
            for key in STATE_KEYS:
                assert np.array_equal(sa[key], sb[key]), (seg, key)
    F.fb_destroy(a)
    F.fb_destroy(b)


def test_fp32_three_level_first_top_draw(oracle_lib):
    """FP32 mode: the first sweep's top-level draws use only the shared
    hyperparameters, so b and psi match the oracle's; the chain then runs 300
    sweeps with finite b and psi and no error."""
    F, g, tops = _pair(oracle_lib, precision=1, burnin=100)
    tops[0].sweep(1)
    F.fb_sweep(g, 1)
    t = F.fb_get_top(g, 0)
    np.testing.assert_allclose(t["b"], tops[0].b, rtol=1e-12)
    np.testing.assert_allclose(t["psi"], tops[0].psi, rtol=1e-12, atol=1e-14)
    F.fb_sweep(g, 300)
    F.fb_sync(g)
    t = F.fb_get_top(g, 0)
    assert np.isfinite(t["b"]) and t["b"] > 0 and np.all(np.isfinite(t["psi"]))
    assert np.all(np.isfinite(t["mean"]))
    F.fb_destroy(g)


def test_top_level_argument_errors():
    F = require_gpu()
    dss = _datasets()
    opts = F.fb_default_options(burnin=5, tune_start=1, precision=0)
    g = F.fb_create_batch([dict(counts=d.y, X=d.X, h=d.h, seed=1 + k) for k, d in enumerate(dss)], opts)
    with pytest.raises(F.FbError):
        F.fb_get_top(g, 0)                                  # no top level yet
    with pytest.raises(F.FbError):
        F.fb_set_top_level(g, -1.0, 1.0, np.ones(2), 0, 3)  # a_b <= 0
    F.fb_set_top_level(g, 1.0, 1.0, np.ones(2), 0, 3)
    with pytest.raises(F.FbError):
        F.fb_get_top(g, 1)                                  # one chain
    F.fb_sweep(g, 6)
    with pytest.raises(F.FbError):
        F.fb_set_top_level(g, 1.0, 1.0, np.ones(2), 0, 3)   # after burn-in
    F.fb_destroy(g)
    # different L across datasets
    two = datagen.small_two_group(G=50, seed=1)
    one = datagen.simulate(50, np.ones((4, 1)), [2.0], [1.0], seed=2)
    g = F.fb_create_batch([dict(counts=two.y, X=two.X, h=two.h, seed=1),
                           dict(counts=one.y, X=one.X, h=one.h, seed=2)], opts)
    with pytest.raises(F.FbError):
        F.fb_set_top_level(g, 1.0, 1.0, np.ones(2), 0, 3)
    F.fb_destroy(g)


@pytest.mark.parametrize("precision", [0, 1])
def test_top_level_at_the_two_level_priors_reproduces_the_two_level_chain(precision):
    """A top level held at b = the datasets' prior rate and psi = 0 (mask 0)
    changes nothing: the chain equals the two-level context's bit for bit."""
    F = require_gpu()
    dss = _datasets()
    opts = F.fb_default_options(burnin=10, tune_start=2, precision=precision, jitter=0, chains=2)
    spec = [dict(counts=d.y, X=d.X, h=d.h, seed=40 + k) for k, d in enumerate(dss)]
    a = F.fb_create_batch(spec, opts)
    b = F.fb_create_batch(spec, opts)
    F.fb_set_top_level(b, 2.0, 3.0, np.array([1.0, 1.0]), 9, 0)
    F.fb_sweep(a, 25)
    F.fb_sweep(b, 25)
    for seg in range(F.fb_num_segments(a)):
        sa, sb = F.fb_get_state(a, seg), F.fb_get_state(b, seg)
        for key in STATE_KEYS:
            assert np.array_equal(sa[key], sb[key]), (seg, key)
    t = F.fb_get_top(b, 1)
    assert t["b"] == 1.0 and np.all(t["psi"] == 0.0)
    F.fb_destroy(a)
    F.fb_destroy(b)
