"""Exact conjugate draws of gamma_g, tau and sigma_l^2 (update_mask bit 12)
on the GPU against the oracle (GPU only).

* FP64: 100 free-running sweeps from a shared state, every draw within a
  relative 1e-5 and every per-draw record identical -- (-1, 0, 0, attempts)
  for an exact draw, the slice counters where a draw fell back.
* Edge cases: shapes below one (N = 1), sigma^2 with G = 1 (shape 0, always
  the slice step), a truncation s_l that binds (frequent fall-backs), L = 7,
  the paper's N = 16 design, exact draws with the shift step.
* FP32 re-synchronised sweeps at the paper design, also at G = 50,000.
* Batched segments equal single runs.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import STATE_KEYS, require_gpu, say
from tests.test_gpu_parity import _compare_fp64, _fp32_resync, _make_pair

pytestmark = pytest.mark.gpu

EXACT = 1 << 12
SHIFT = 1 << 11


def test_fp64_parity_100_sweeps_exact(oracle_lib):
    ds = datagen.small_two_group(G=1000, seed=0)
    F, g, o = _make_pair(oracle_lib, ds, seed=13, burnin=40, tune_start=5, precision=0,
                         update_mask=0xFE | EXACT)
    F.fb_set_state(g, o.get_state())
    for it in range(100):
        assert o.sweep(1) == 0
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"exact sweep {it + 1}")
    cg = F.fb_debug_counts(g)
    assert np.all(cg["gam"][:, 0] == -1) and np.all(cg["hyp"][[1, 2 + 0, 2 + 1], 0] == -1)
    mo, mg = o.moments(), F.fb_summaries(g)
    for k in ("mean_gam", "msq_gam", "mean_hyp", "msq_hyp", "mean_beta"):
        np.testing.assert_allclose(mg[k], mo[k], rtol=1e-9, atol=1e-12, err_msg=k)
    F.fb_destroy(g)


def _edge():
    two = datagen.design_two_groups(2)
    H2 = np.array([[1.0, 1.0], [1.0, -1.0]])
    H8 = np.kron(np.kron(H2, H2), H2)[:, :7]
    return [
        ("G1", datagen.simulate(1, two, [3.0, 0.0], [1.5, 0.5], seed=1), {}),
        ("N1_L1", datagen.simulate(100, np.ones((1, 1)), [1.0], [1.0], seed=5), {}),
        ("G65_ragged", datagen.simulate(65, two, [3.0, 0.0], [1.5, 0.5], seed=2), {}),
        ("tight_s", datagen.simulate(150, two, [3.0, 0.0], [1.5, 0.5], seed=12),
         dict(priors=dict(a=2.0, b=0.5, d=50.0, c=[3.0, 1.0], s=[5.0, 0.42]))),
        ("paper_N16", datagen.paper_design_16(G=300, seed=8), {}),
        ("L7_N8", datagen.simulate(90, H8, [3.0] + [0.0] * 6, [1.5] + [0.3] * 6, seed=13), {}),
        ("paper_N16_shift", datagen.paper_design_16(G=300, seed=9), dict(update_mask=0xFE | EXACT | SHIFT)),
    ]


@pytest.mark.parametrize("name,ds,kw", _edge(), ids=[e[0] for e in _edge()])
def test_fp64_parity_edge_cases_exact(oracle_lib, name, ds, kw):
    say("exact edge case", name, ds.y.shape)
    kw = dict(kw)
    kw.setdefault("update_mask", 0xFE | EXACT)
    ora_kw = {}
    if "priors" in kw:
        p = kw["priors"]
        ora_kw = dict(a=p["a"], b=p["b"], d=p["d"], c=np.array(p["c"]), s=np.array(p["s"]))
    F, g, o = _make_pair(oracle_lib, ds, seed=4, burnin=10, tune_start=2, precision=0, **kw, **ora_kw)
    F.fb_set_state(g, o.get_state())
    n_fallback = 0
    for it in range(30):
        o.sweep(1)
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"{name} sweep {it + 1}")
        n_fallback += int((o.counts()["hyp"][2:, 0] >= 0).sum())
    if name == "tight_s":
        assert n_fallback > 0          # the slice step took over for sigma^2 at least once
    if name == "G1":
        assert n_fallback == 30 * ds.L  # shape (G - 1)/2 = 0: always the slice step
    F.fb_destroy(g)


def test_fp64_parity_shapes_below_one(oracle_lib):
    """N = 1 and nu held at 0.01 give gamma_g the shape 0.505 and, with a = 0.2
    and G = 65, tau the shape 0.525: both take the U^(1/alpha) path."""
    ds = datagen.simulate(65, np.ones((1, 1)), [1.0], [1.0], seed=5)
    mask = (0xFE & ~(1 << 3)) | EXACT
    F, g, o = _make_pair(oracle_lib, ds, seed=4, burnin=10, tune_start=2, precision=0, update_mask=mask,
                         priors=dict(a=0.2, b=1.0, d=1000.0, c=[10.0], s=[100.0]), a=0.2, b=1.0)
    st = o.get_state()
    st["hyp"][0] = 0.01
    o.set_state(st)
    F.fb_set_state(g, o.get_state())
    for it in range(30):
        assert o.sweep(1) == 0
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"shape < 1 sweep {it + 1}")
    F.fb_destroy(g)


def test_fp32_parity_resync_exact(oracle_lib):
    ds = datagen.paper_design_16(G=2000, seed=0)
    frac, worst = _fp32_resync(oracle_lib, ds, seed=23, n_sweeps=60, warm=40, label="fp32 exact G=2000",
                               update_mask=0xFE | EXACT)
    assert frac < 2e-3
    assert worst < 1e-2


def test_fp32_parity_full_size_exact(oracle_lib):
    """G = 50,000, N = 16, L = 5 in the default launch configuration.  (The
    shift step in FP32 has a parity test of its own, with a tolerance on the
    conditional's scale; these re-synchronised sweeps take the slice-step
    tolerance.)"""
    ds = datagen.paper_design_16(G=50_000, seed=0)
    frac, worst = _fp32_resync(oracle_lib, ds, seed=1, n_sweeps=3, warm=8, threads=16,
                               label="fp32 exact G=50000", update_mask=0xFE | EXACT)
    assert frac < 2e-3
    assert worst < 1e-2


@pytest.mark.parametrize("precision", [0, 1])
def test_exact_batched_segments_match_single_runs(precision):
    F = require_gpu()
    meta = [(300, 4), (1000, 16), (77, 8)]
    dss = [datagen.batched_dataset(k + 1, G, N) for k, (G, N) in enumerate(meta)]
    opts = dict(burnin=8, tune_start=2, precision=precision, jitter=1, chains=2, debug_counts=1,
                update_mask=0xFE | EXACT)
    b = F.fb_create_batch([dict(counts=d.y, X=d.X, h=d.h, seed=300 + k) for k, d in enumerate(dss)],
                          F.fb_default_options(**opts))
    F.fb_sweep(b, 20)
    for k, d in enumerate(dss):
        one = F.fb_create(d.y, d.X, d.h, seed=300 + k, options=F.fb_default_options(**opts))
        F.fb_sweep(one, 20)
        for ch in range(2):
            sa, sb = F.fb_get_state(b, 2 * k + ch), F.fb_get_state(one, ch)
            for key in STATE_KEYS:
                assert np.array_equal(sa[key], sb[key]), (k, ch, key)
        F.fb_destroy(one)
    F.fb_destroy(b)
