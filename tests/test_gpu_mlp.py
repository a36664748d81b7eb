"""The learned beta proposal on the GPU (matrix-core network, training, IMH).

* The 32x32x16 BF16 matrix-core product matches numpy exactly on inputs whose
  products and sums are exact in FP32 (checks the lane layout).
* The network's outputs (proposal mean, log-diagonal and lower triangle of
  its factor) and the training gradients match the FP64 oracle on the same
  BF16-rounded weights and inputs (BF16 activations on the GPU: per-tensor
  relative error <= 2e-2, cosine > 0.999).
* The features of every gene match the oracle's.
* A full sweep with the IMH beta step (Laplace approximation corrected by a
  shift, a scale and a correlated factor) matches the oracle draw for draw in
  FP64 when the network's outputs are exact (a network with zero weights and
  biases on a 1/64 grid).
* Training on pairs collected from the plain sampler lowers the loss.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import require_gpu, say
from tests.test_oracle_mlp import constant_model, random_model

pytestmark = pytest.mark.gpu


def bf16(x):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def to_gpu_params(m, L):
    """Oracle model dict -> the library's padded FP32 parameter dict."""
    from paper_1606_06659_amd import fbmc
    p = fbmc.mlp_zeros()
    p["fmean"][:] = m["fmean"]
    p["fscale"][:] = m["fscale"]
    p["W1"][:] = m["W1"]
    p["b1"][:] = m["b1"]
    p["W2"][:] = m["W2"]
    p["b2"][:] = m["b2"]
    O = fbmc.mlp_outputs(L)
    p["W3"][:, :O] = m["W3"]
    p["b3"][:O] = m["b3"]
    p["omean"][:L] = m["omean"]
    p["oscale"][:L] = m["oscale"]
    return p


def rounded_oracle_model(m):
    """The oracle's view of what the GPU multiplies: BF16 weights, FP32 rest."""
    r = dict(m)
    for k in ("W1", "W2", "W3"):
        r[k] = bf16(m[k])
    for k in ("b1", "b2", "b3", "fmean", "fscale", "omean", "oscale"):
        r[k] = np.asarray(m[k], np.float32).astype(np.float64)
    return r


def test_mfma_lane_layout():
    F = require_gpu()
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 9, size=(32, 16)).astype(np.float32) / 4
    B = rng.integers(-8, 9, size=(16, 32)).astype(np.float32) / 8
    C = F.fb_mfma_probe(A, B)
    assert np.array_equal(C, (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32))


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _cos(a, b):
    a, b = a.ravel(), b.ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def test_mlp_forward_matches_oracle(oracle_lib):
    F = require_gpu()
    rng = np.random.default_rng(1)
    L = 5
    m = random_model(rng, L)
    phi = rng.normal(0, 1.5, (300, 32))
    mu_g, ls_g, off_g = F.fb_mlp_forward(to_gpu_params(m, L), L, phi)
    mr = rounded_oracle_model(m)
    x = bf16(np.clip((phi.astype(np.float32) - mr["fmean"].astype(np.float32)) * mr["fscale"].astype(np.float32),
                     np.float32(-8), np.float32(8)))
    # feed the oracle the rounded standardised inputs through an identity standardisation
    mo = dict(mr, fmean=np.zeros(32), fscale=np.ones(32))
    mu_o, ls_o, off_o = oracle_lib.mlp_forward(mo, x)
    for name, g, o in (("mu", mu_g, mu_o), ("ls", ls_g, ls_o), ("off", off_g, off_o)):
        say(name, "rel", _rel(g, o), "cos", _cos(g - g.mean(0), o - o.mean(0)))
        assert _rel(g, o) < 2e-2, _rel(g, o)
        assert _cos(g - g.mean(0), o - o.mean(0)) > 0.999


def conditioned_model(rng, L):
    """A random network whose factor stays well conditioned (small strict
    lower triangle), so BF16 rounding is not amplified by the triangular solve."""
    m = random_model(rng, L)
    m["W3"][:, L:2 * L] *= 0.3
    m["W3"][:, 2 * L:] *= 0.1
    m["b3"][2 * L:] *= 0.1
    return m


def test_mlp_gradients_match_oracle(oracle_lib):
    F = require_gpu()
    rng = np.random.default_rng(2)
    L = 5
    m = conditioned_model(rng, L)
    B = 256
    phi = rng.normal(0, 1.5, (B, 32))
    tgt = rng.normal(0, 1, (B, L))
    loss_g, grads_g = F.fb_mlp_loss_grad(to_gpu_params(m, L), L, phi, tgt)
    mr = rounded_oracle_model(m)
    x = bf16(np.clip((phi.astype(np.float32) - mr["fmean"].astype(np.float32)) * mr["fscale"].astype(np.float32),
                     np.float32(-8), np.float32(8)))
    mo = dict(mr, fmean=np.zeros(32), fscale=np.ones(32))
    loss_o, grads_o = oracle_lib.mlp_loss_grad(mo, x, tgt.astype(np.float32))
    assert abs(loss_g - loss_o) < 2e-2 * max(1.0, abs(loss_o)), (loss_g, loss_o)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        O = F.mlp_outputs(L)
        g = grads_g[k][:, :O] if k == "W3" else (grads_g[k][:O] if k == "b3" else grads_g[k])
        o = grads_o[k]
        say(k, "rel", _rel(g, o), "cos", _cos(g, o))
        assert _rel(g, o) < 2e-2, (k, _rel(g, o))
        assert _cos(g, o) > 0.999, (k, _cos(g, o))
    O = F.mlp_outputs(L)
    assert np.all(grads_g["W3"][:, O:] == 0) and np.all(grads_g["b3"][O:] == 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_features_match_oracle(oracle_lib, precision):
    F = require_gpu()
    ds = datagen.paper_design_16(G=700, seed=3)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=5, burnin=20, tune_start=2)
    o.sweep(30)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=5, options=F.fb_default_options(precision=precision, jitter=0))
    F.fb_set_state(g, o.get_state())
    got = F.fb_features(g).astype(np.float64)
    want = o.features(32)
    F.fb_destroy(g)
    tol = 1e-9 if precision == 0 else 3e-5
    # float features are computed from a float state: compare relative to scale
    assert np.max(np.abs(got - want) / (np.abs(want) + 1.0)) < max(tol, 1e-6), np.max(np.abs(got - want))


def test_imh_sweep_parity_fp64(oracle_lib):
    """Every gene takes the IMH step; a zero-weight network makes the proposal
    exact on both sides, so the whole sweep matches draw for draw."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=500, seed=4)
    L = ds.L
    # a correction of the Laplace proposal in its whitened coordinates: mean
    # shift, scale and a correlated factor, on a 1/64 grid (exact in FP32)
    mu = np.round(np.random.default_rng(11).uniform(-0.4, 0.4, L) * 64) / 64
    log_s = np.round(np.full(L, np.log(0.9)) * 64) / 64
    off = np.round(np.random.default_rng(12).uniform(-0.3, 0.3, L * (L - 1) // 2) * 64) / 64
    m = constant_model(L, mu, log_s, off=off)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=9, burnin=10, tune_start=2)
    o.sweep(15)
    opts = F.fb_default_options(precision=0, jitter=0, debug_counts=1, burnin=10, tune_start=2)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=9, options=opts)
    F.fb_set_state(g, o.get_state())
    F.fb_proposal_set(g, to_gpu_params(m, L))
    F.fb_fallback(g, 0, np.zeros(ds.G, np.int32))
    F.fb_set_beta_update(g, F.FB_BETA_LEARNED)
    o.set_proposal(m, np.zeros(ds.G, np.int32))
    n_acc = 0
    acc_gene = np.zeros(ds.G, np.int64)
    for it in range(20):
        o.sweep(1)
        F.fb_sweep(g, 1)
        so, sg = o.get_state(), F.fb_get_state(g)
        acc_o, la_o = o.imh()
        acc_g = F.fb_imh_last(g)
        flips = np.flatnonzero(acc_o != acc_g)
        assert flips.size == 0, (it, flips[:5], la_o[flips[:5]])
        n_acc += int(np.sum(acc_o == 1))
        acc_gene += acc_o == 1
        for k in ("eps", "gam", "beta", "hyp"):
            np.testing.assert_allclose(sg[k], so[k], rtol=1e-9, atol=1e-12, err_msg=f"sweep {it} {k}")
    assert 0 < n_acc < 20 * ds.G
    # acceptance statistics: all 20 sweeps are past burn-in, every gene took the IMH step
    sm = F.fb_summaries(g)
    assert np.all(sm["imh_steps"] == 20)
    assert np.array_equal(sm["imh_accepts"], acc_gene)
    F.fb_destroy(g)


@pytest.mark.parametrize("shift", [0, 1])
def test_imh_sweep_parity_with_fallback_genes_fp64(oracle_lib, shift):
    """As above with about 30% of the genes flagged for fallback: they take
    the slice steps in their own groups, the others the IMH step, and the whole
    sweep (moments and reductions included) matches the oracle; with the shift
    step on, it follows both kinds of beta step."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=700, seed=8)
    L = ds.L
    mu = np.round(np.random.default_rng(15).uniform(-0.4, 0.4, L) * 64) / 64
    log_s = np.round(np.full(L, np.log(1.1)) * 64) / 64
    off = np.round(np.random.default_rng(13).uniform(-0.3, 0.3, L * (L - 1) // 2) * 64) / 64
    m = constant_model(L, mu, log_s, off=off)
    mask = (np.random.default_rng(14).uniform(size=ds.G) < 0.3).astype(np.int32)
    upd = F.FB_UPDATE_ALL | (F.FB_SHIFT if shift else 0)
    # hand the state over before the end of burn-in, so that both sides
    # accumulate the running moments over the same post-burn-in sweeps
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=19, burnin=10, tune_start=2, update_mask=upd)
    o.sweep(7)
    opts = F.fb_default_options(precision=0, jitter=0, debug_counts=1, burnin=10, tune_start=2,
                                update_mask=upd)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=19, options=opts)
    F.fb_set_state(g, o.get_state())
    F.fb_proposal_set(g, to_gpu_params(m, L))
    F.fb_fallback(g, 0, mask)
    F.fb_set_beta_update(g, F.FB_BETA_LEARNED)
    o.set_proposal(m, mask)
    steps, accepts = np.zeros(ds.G, np.int64), np.zeros(ds.G, np.int64)
    for it in range(12):
        o.sweep(1)
        F.fb_sweep(g, 1)
        so, sg = o.get_state(), F.fb_get_state(g)
        acc_o, _ = o.imh()
        acc_g = F.fb_imh_last(g)
        assert np.array_equal(acc_o, acc_g), (it, np.flatnonzero(acc_o != acc_g)[:5])
        assert np.all(acc_g[mask == 1] == -1) and np.all(acc_g[mask == 0] >= 0)
        if 8 + it > 10:          # sweeps m > M_B count toward the acceptance statistics
            steps += acc_o >= 0
            accepts += acc_o == 1
        for k in ("eps", "gam", "beta", "hyp", "w_beta", "waux_beta"):
            np.testing.assert_allclose(sg[k], so[k], rtol=1e-9, atol=1e-12, err_msg=f"sweep {it} {k}")
        np.testing.assert_allclose(F.fb_reductions(g), o.reductions(), rtol=1e-9, atol=1e-9)
    sm, om = F.fb_summaries(g), o.moments()
    np.testing.assert_allclose(sm["mean_beta"], om["mean_beta"], rtol=1e-9, atol=1e-12)
    # the oracle's decisions over the sampling sweeps; fallback genes take no IMH step
    assert np.array_equal(sm["imh_steps"], steps) and np.array_equal(sm["imh_accepts"], accepts)
    assert np.all(steps[mask == 1] == 0) and np.all(steps[mask == 0] == 9)
    # back to burn-in: the counts restart
    st = F.fb_get_state(g)
    st["m"] = 5
    F.fb_set_state(g, st)
    assert not F.fb_summaries(g)["imh_steps"].any()
    F.fb_destroy(g)


@pytest.mark.parametrize("precision", [0, 1])
def test_laplace_mode_equals_zero_network(precision):
    """FB_BETA_LAPLACE (no network kernel) and FB_BETA_LEARNED with a network
    whose outputs are all zero (omean 0, oscale 1) propose the same Laplace
    base, so the chains agree bit for bit, fallback genes included."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=900, seed=21)
    L = ds.L
    opts = F.fb_default_options(precision=precision, jitter=0, burnin=10, tune_start=2)
    mask = (np.random.default_rng(22).uniform(size=ds.G) < 0.2).astype(np.int32)
    ctx = []
    for mode in ("laplace", "zero_net"):
        g = F.fb_create(ds.y, ds.X, ds.h, seed=23, options=opts)
        F.fb_sweep(g, 6)
        if mode == "zero_net":
            F.fb_proposal_set(g, to_gpu_params(constant_model(L, np.zeros(L), np.zeros(L)), L))
            F.fb_set_beta_update(g, F.FB_BETA_LEARNED)
        else:
            F.fb_set_beta_update(g, F.FB_BETA_LAPLACE)
        F.fb_fallback(g, 0, mask)
        ctx.append(g)
    for n in (5, 9):
        for g in ctx:
            F.fb_sweep(g, n)
        sa, sb = F.fb_get_state(ctx[0]), F.fb_get_state(ctx[1])
        for k in ("eps", "gam", "beta", "hyp"):
            assert np.array_equal(sa[k], sb[k]), (n, k)
        assert np.array_equal(F.fb_imh_last(ctx[0]), F.fb_imh_last(ctx[1]))
    last = F.fb_imh_last(ctx[0])
    assert np.all(last[mask == 1] == -1) and np.all(last[mask == 0] >= 0)
    for g in ctx:
        F.fb_destroy(g)


@pytest.mark.parametrize("shift,frac", [(0, 0.25), (1, 0.25), (1, 0.0)])
def test_laplace_mode_parity_fp64(oracle_lib, shift, frac):
    """The Laplace-only proposal against the oracle's IMH step with a
    zero-output network, with fallback genes (their slice steps in groups of
    their own) or none (with the shift step: the fused MH and shift kernel),
    optionally with the shift step."""
    F = require_gpu()
    ds = datagen.paper_design_16(G=600, seed=24)
    L = ds.L
    m = constant_model(L, np.zeros(L), np.zeros(L))
    mask = (np.random.default_rng(25).uniform(size=ds.G) < frac).astype(np.int32)
    upd = F.FB_UPDATE_ALL | (F.FB_SHIFT if shift else 0)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=26, burnin=10, tune_start=2, update_mask=upd)
    o.sweep(7)
    opts = F.fb_default_options(precision=0, jitter=0, debug_counts=1, burnin=10, tune_start=2,
                                update_mask=upd)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=26, options=opts)
    F.fb_set_state(g, o.get_state())
    F.fb_set_beta_update(g, F.FB_BETA_LAPLACE)
    F.fb_fallback(g, 0, mask)
    o.set_proposal(m, mask)
    n_acc = 0
    for it in range(12):
        o.sweep(1)
        F.fb_sweep(g, 1)
        so, sg = o.get_state(), F.fb_get_state(g)
        acc_o, _ = o.imh()
        acc_g = F.fb_imh_last(g)
        assert np.array_equal(acc_o, acc_g), (it, np.flatnonzero(acc_o != acc_g)[:5])
        n_acc += int(np.sum(acc_g == 1))
        for k in ("eps", "gam", "beta", "hyp"):
            np.testing.assert_allclose(sg[k], so[k], rtol=1e-9, atol=1e-12, err_msg=f"sweep {it} {k}")
    assert 0 < n_acc < 12 * int((mask == 0).sum())
    sm, om = F.fb_summaries(g), o.moments()
    np.testing.assert_allclose(sm["mean_beta"], om["mean_beta"], rtol=1e-9, atol=1e-12)
    F.fb_destroy(g)


def test_laplace_calibration_needs_no_network():
    F = require_gpu()
    ds = datagen.paper_design_16(G=800, seed=27)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=28, options=F.fb_default_options(precision=1, burnin=200,
                                                                            tune_start=20))
    F.fb_sweep(g, 100)
    with pytest.raises(F.FbError):
        F.fb_proposal_calibrate(g, 20, 0.2)          # the network's proposal: no network yet
    F.fb_set_beta_update(g, F.FB_BETA_LAPLACE)
    F.fb_proposal_calibrate(g, 40, 0.2)
    fb = F.fb_fallback(g)
    assert set(np.unique(fb)) <= {0, 1}
    F.fb_sweep(g, 20)
    last = F.fb_imh_last(g)
    assert np.all(last[fb == 1] == -1) and np.all(last[fb == 0] >= 0)
    say("laplace calibration: fallback fraction", fb.mean(), "acceptance", np.mean(last[fb == 0] == 1))
    F.fb_destroy(g)


def test_training_lowers_loss():
    F = require_gpu()
    ds = datagen.small_two_group(G=2000, seed=6)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=3, options=F.fb_default_options(precision=1, burnin=200,
                                                                             tune_start=20, jitter=0))
    F.fb_sweep(g, 200)
    F.fb_proposal_collect(g, 20, every=2)
    losses = F.fb_proposal_train(g, F.fb_default_train_opts(epochs=40))
    say("training losses", losses[:3], losses[-3:])
    assert np.all(np.isfinite(losses))
    # the targets are whitened by the Laplace approximation, so the untrained
    # network (a small correction) already starts near L / 2 = 1
    assert losses[-1] < losses[0]
    params = F.fb_proposal_get(g)
    assert np.all(np.isfinite(params["W1"]))
    F.fb_proposal_calibrate(g, 20, 0.2)
    F.fb_set_beta_update(g, F.FB_BETA_LEARNED)
    F.fb_sweep(g, 50)
    last = F.fb_imh_last(g)
    fb = F.fb_fallback(g)
    say("fallback genes", int(fb.sum()), "accept rate", float(np.mean(last[fb == 0] == 1)))
    assert np.all(last[fb == 1] == -1)
    assert np.mean(last[fb == 0] == 1) > 0.6
    assert fb.mean() < 0.05
    F.fb_destroy(g)
