"""Parity of the HIP shift step with the FP64 oracle (GPU only).

The shift step moves beta_g -> beta_g + delta, eps_g -> eps_g - X delta with
delta drawn exactly from its Gaussian conditional (an addition to Algorithm 1
that keeps eps_g + X beta_g).

* FP64: 60 free-running sweeps of the full chain with the step on, every draw,
  width, integer record, reduction and running moment as in the plain FP64
  parity test.
* FP32: one shift step from a shared state; delta agrees with the oracle's to
  1e-4 of the conditional standard deviation of each coefficient (the FP32
  rounding of the L x L Cholesky factor and solves), and eps + X beta is kept
  to FP32 rounding.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import require_gpu, say
from tests.test_gpu_parity import _compare_fp64, _make_pair

pytestmark = pytest.mark.gpu


def _mask(F, oracle_lib):
    assert F.FB_SHIFT == 1 << 11 and F.FB_UPDATE_ALL == oracle_lib.UPDATE_ALL
    return F.FB_UPDATE_ALL | F.FB_SHIFT


@pytest.mark.parametrize("which", ["two_group", "paper"])
def test_fp64_parity_with_shift_step(oracle_lib, which):
    F = require_gpu()
    ds = (datagen.small_two_group(G=1000, seed=0) if which == "two_group"
          else datagen.paper_design_16(G=700, seed=3))
    mask = _mask(F, oracle_lib)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=13, burnin=25, tune_start=4, update_mask=mask)
    opts = F.fb_default_options(burnin=25, tune_start=4, precision=0, debug_counts=1, jitter=0,
                                update_mask=mask, thin=1, trace_genes=7, trace_capacity=80)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=13, options=opts)
    F.fb_set_state(g, o.get_state())
    for it in range(60):
        assert o.sweep(1) == 0
        F.fb_sweep(g, 1)
        _compare_fp64(F, g, o, f"{which} sweep {it + 1}")
        np.testing.assert_allclose(F.fb_reductions(g), o.reductions(), rtol=1e-9, atol=1e-9)
    mo, mg = o.moments(), F.fb_summaries(g)
    assert mg["count"] == mo["count"] == 35
    for k in ("mean_eps", "msq_eps", "mean_gam", "msq_gam", "mean_beta", "msq_beta", "mean_hyp", "msq_hyp"):
        np.testing.assert_allclose(mg[k], mo[k], rtol=1e-9, atol=1e-12, err_msg=k)
    # the traced beta is the state after the shift
    tr, _ = F.fb_trace(g)
    genes = F.fb_trace_genes(g)
    L = ds.L
    last = tr[-1]
    np.testing.assert_allclose(last[2 + 2 * L:].reshape(-1, L + 1)[:, 1:], o.get_state()["beta"][genes],
                               rtol=1e-6, atol=1e-7)
    F.fb_destroy(g)


def test_fp32_shift_step_matches_oracle(oracle_lib):
    F = require_gpu()
    ds = datagen.paper_design_16(G=3000, seed=9)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=17, burnin=20, tune_start=2)
    o.sweep(30)
    st0 = o.get_state()
    shift = F.FB_SHIFT
    o.set_update_mask(shift)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=17,
                    options=F.fb_default_options(burnin=20, tune_start=2, precision=1, jitter=0,
                                                 update_mask=shift))
    F.fb_set_state(g, st0)
    assert o.sweep(1) == 0
    F.fb_sweep(g, 1)
    so, sg = o.get_state(), F.fb_get_state(g)
    X, L = ds.X, ds.L
    s2 = st0["hyp"][2 + L:]
    d_o = so["beta"] - st0["beta"]
    d_g = sg["beta"].astype(np.float64) - st0["beta"].astype(np.float32).astype(np.float64)
    # conditional standard deviations: sqrt(diag(P^-1)), P = X^T X / gamma + diag(1 / sigma^2)
    P = (X.T @ X)[None] / st0["gam"][:, None, None] + np.diag(1.0 / s2)[None]
    sd = np.sqrt(np.diagonal(np.linalg.inv(P), axis1=1, axis2=2))
    err = np.abs(d_g - d_o) / sd
    say("fp32 shift: max |delta error| / sd", err.max(), "median", np.median(err))
    assert err.max() < 1e-4, err.max()
    z0 = st0["eps"] + st0["beta"] @ X.T
    z1 = sg["eps"].astype(np.float64) + sg["beta"].astype(np.float64) @ X.T
    assert np.max(np.abs(z1 - z0) / (np.abs(z0) + 1.0)) < 1e-5
    np.testing.assert_array_equal(sg["hyp"], so["hyp"])
    F.fb_destroy(g)


@pytest.mark.parametrize("precision,beta", [(0, "slice"), (1, "slice"), (0, "laplace"), (1, "laplace")])
def test_fused_and_separate_shift_kernels_agree(precision, beta):
    """The shift step inside the gamma/beta kernel (the default) and in a
    kernel of its own give the same chain bit for bit, also under graph replay
    and with events, trace and moments on; with the slice steps and with the
    independence-MH beta step (Laplace proposal, no fallback genes)."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=1500, seed=4)
    opts = F.fb_default_options(burnin=15, tune_start=3, precision=precision, jitter=0,
                                update_mask=F.FB_UPDATE_ALL | F.FB_SHIFT, thin=1, trace_genes=9,
                                trace_capacity=60)
    a = F.fb_create(ds.y, ds.X, ds.h, seed=21, options=opts)
    b = F.fb_create(ds.y, ds.X, ds.h, seed=21, options=opts)
    F.fb_set_shift_fusion(b, False)
    ev = [[(np.array([0.0, 2.0, 0.0, 1.0, 0.0]), 0.0)]]
    for g in (a, b):
        F.fb_set_contrasts(g, ev, 5)
        if beta == "laplace":
            F.fb_set_beta_update(g, F.FB_BETA_LAPLACE)
            F.fb_fallback(g, 0, np.zeros(ds.G, np.int32))
    for i, n in enumerate((12, 9, 20)):
        if i == 2:
            F.fb_set_graph(a, 5)
            F.fb_set_graph(b, 5)
        say("fused vs separate shift kernel: sweeps", n, "precision", precision)
        F.fb_sweep(a, n)
        F.fb_sweep(b, n)
        sa, sb = F.fb_get_state(a), F.fb_get_state(b)
        for k in ("eps", "gam", "beta", "hyp", "w_eps", "w_beta"):
            assert np.array_equal(sa[k], sb[k]), (i, k)
        ma, mb = F.fb_summaries(a), F.fb_summaries(b)
        for k in ma:
            assert np.array_equal(np.asarray(ma[k]), np.asarray(mb[k])), (i, k)
        assert np.array_equal(F.fb_trace(a)[0], F.fb_trace(b)[0])
        assert np.array_equal(F.fb_event_counts(a, 1)[0], F.fb_event_counts(b, 1)[0])
        if beta == "laplace":
            assert np.array_equal(F.fb_imh_last(a), F.fb_imh_last(b))
            assert np.all(F.fb_imh_last(a) >= 0)
    F.fb_destroy(a)
    F.fb_destroy(b)
