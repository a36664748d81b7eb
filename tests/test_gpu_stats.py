"""Long-run agreement of the GPU sampler (FP32 log densities) with the FP64
oracle on the G = 1000, N = 4 two-group workload, 2000 iterations (GPU only).

The two chains use different seeds, so they are independent draws of the same
posterior; their posterior means must agree within Monte Carlo error by the
criteria of tests/chain_compare.py (calibrated on two oracle chains, with power
shown against a planted mistake on the CPU).  The device's running moments
(Welford, FP64) must equal the means of the traced draws.
"""
import os

import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.chain_compare import agree, agree_3mcse, compare
from tests.gpu_common import require_gpu, say
from tests.test_oracle_chains import BURNIN, ITERS, oracle_draws

pytestmark = pytest.mark.gpu


def test_posterior_means_within_mcse(oracle_lib):
    F = require_gpu()
    ds = datagen.small_two_group(G=1000, seed=0)
    G, L = ds.G, ds.L
    post = ITERS - BURNIN
    say("oracle chain", ITERS, "sweeps")
    a = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=21, burnin=BURNIN, tune_start=BURNIN // 10,
                                       threads=min(8, os.cpu_count() or 1)), ds)
    say("gpu chain", ITERS, "sweeps")
    opts = F.fb_default_options(burnin=BURNIN, tune_start=BURNIN // 10, precision=1, jitter=0, thin=1,
                                trace_genes=G, trace_after_burnin=1, trace_capacity=post)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=22, options=opts)
    F.fb_sweep(g, ITERS)
    tr, dropped = F.fb_trace(g)
    summ = F.fb_summaries(g)
    F.fb_destroy(g)
    assert tr.shape[0] == post and dropped == 0
    tr = tr.astype(np.float64)
    hyp = tr[:, :2 + 2 * L]
    genes = tr[:, 2 + 2 * L:].reshape(post, G, L + 1)
    gam, beta = genes[:, :, 0], genes[:, :, 1:]

    # the running moments are the means of the draws
    np.testing.assert_allclose(summ["mean_gam"], gam.mean(0), rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(summ["mean_beta"], beta.mean(0), rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(summ["mean_hyp"], hyp.mean(0), rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(summ["msq_beta"], (beta ** 2).mean(0), rtol=2e-5, atol=1e-6)

    r = compare(hyp, gam, beta, *a)
    say("gpu vs oracle", r)
    assert agree(r), r


@pytest.mark.parametrize("form", ["shift_exact", "laplace_shift_exact", "learned_shift_exact",
                                  "three_level_top_fixed"])
def test_other_forms_agree_with_the_oracle(oracle_lib, form):
    """The options that leave the posterior invariant -- the shift step with
    the exact conjugate draws; the same with the Laplace independence step
    (calibrated during burn-in); with the trained network's independence step
    (pairs collected, network trained, fallback calibrated during burn-in); a
    three-level context whose top level is held at the two-level priors
    (b = 1, psi = 0, one group) -- give posterior means within 3 Monte Carlo
    standard errors of an oracle chain's (agree_3mcse).  The oracle chain
    takes the shift step and the exact draws too: over 2,000 sweeps the plain
    chain's sigma^2 has not mixed (two plain oracle chains already differ by
    z = 4.4 in sigma_2^2, and plain against shifted oracle chains by 8), while
    two shifted oracle chains agree to |z| < 3 on every hyperparameter."""
    F = require_gpu()
    ds = datagen.small_two_group(G=1000, seed=0)
    G, L = ds.G, ds.L
    post = ITERS - BURNIN
    mask = F.FB_UPDATE_ALL | F.FB_SHIFT | F.FB_EXACT
    a = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=31, burnin=BURNIN, tune_start=BURNIN // 10,
                                       threads=min(8, os.cpu_count() or 1), update_mask=mask), ds)
    opts = F.fb_default_options(burnin=BURNIN, tune_start=BURNIN // 10, precision=1, jitter=0, thin=1,
                                trace_genes=G, trace_after_burnin=1, trace_capacity=post, update_mask=mask)
    if form == "three_level_top_fixed":
        g = F.fb_create_batch([dict(counts=ds.y, X=ds.X, h=ds.h, seed=32)], opts)
        F.fb_set_top_level(g, 1.0, 1.0, np.full(L, 10.0), 33, 0)
    else:
        g = F.fb_create(ds.y, ds.X, ds.h, seed=32, options=opts)
    say("gpu chain", form, ITERS, "sweeps")
    if form == "laplace_shift_exact":
        F.fb_sweep(g, BURNIN - 300)
        F.fb_set_beta_update(g, F.FB_BETA_LAPLACE)
        F.fb_proposal_calibrate(g, 100, 0.2)
        F.fb_sweep(g, ITERS - (BURNIN - 300) - 100)
        say("laplace fallback fraction", F.fb_fallback(g).mean())
    elif form == "learned_shift_exact":
        F.fb_sweep(g, 150)
        F.fb_proposal_collect(g, 200, every=2)
        losses = F.fb_proposal_train(g, F.fb_default_train_opts(epochs=100))
        F.fb_proposal_calibrate(g, 50, 0.2)
        F.fb_set_beta_update(g, F.FB_BETA_LEARNED)
        F.fb_sweep(g, ITERS - 400)
        last = F.fb_imh_last(g)
        say("learned: loss", losses[0], "->", losses[-1], "fallback fraction", F.fb_fallback(g).mean(),
            "accept", np.mean(last[last >= 0] == 1))
    else:
        F.fb_sweep(g, ITERS)
    tr, dropped = F.fb_trace(g)
    F.fb_destroy(g)
    assert tr.shape[0] == post and dropped == 0
    tr = tr.astype(np.float64)
    hyp = tr[:, :2 + 2 * L]
    genes = tr[:, 2 + 2 * L:].reshape(post, G, L + 1)
    r = compare(hyp, genes[:, :, 0], genes[:, :, 1:], *a)
    say("gpu", form, "vs oracle", r)
    assert agree_3mcse(r), r


def test_rhat_from_device_moments():
    """Section 3.1's convergence check from the device's running moments
    alone: four overdispersed chains (with the shift step and the exact draws,
    which mix fast enough for 1,500 post-burn-in sweeps) give R-hat near 1 for
    the genes and the hyperparameters, and the device moments give the same
    R-hat as the traced draws of the traced genes."""
    from paper_1606_06659_amd import diagnostics
    F = require_gpu()
    ds = datagen.small_two_group(G=1000, seed=0)
    G, L, C = ds.G, ds.L, 4
    post = ITERS - BURNIN
    T = 50
    opts = F.fb_default_options(burnin=BURNIN, tune_start=BURNIN // 10, precision=1, jitter=1, chains=C, thin=1,
                                trace_genes=T, trace_after_burnin=1, trace_capacity=post,
                                update_mask=F.FB_UPDATE_ALL | F.FB_SHIFT | F.FB_EXACT)
    g = F.fb_create(ds.y, ds.X, ds.h, seed=61, options=opts)
    F.fb_sweep(g, ITERS)
    summ = [F.fb_summaries(g, c) for c in range(C)]
    traces = [F.fb_trace(g, c)[0].astype(np.float64) for c in range(C)]
    genes = F.fb_trace_genes(g)
    F.fb_destroy(g)
    assert all(s["count"] == post for s in summ)
    st = lambda k: np.stack([s[k] for s in summ])
    r_beta = diagnostics.rhat_from_moments(st("mean_beta"), st("msq_beta"), post)
    r_gam = diagnostics.rhat_from_moments(st("mean_gam"), st("msq_gam"), post)
    r_hyp = diagnostics.rhat_from_moments(st("mean_hyp"), st("msq_hyp"), post)
    say("R-hat: beta 99th pct", np.percentile(r_beta, 99), "gamma 99th pct", np.percentile(r_gam, 99),
        "hyper max", r_hyp.max())
    assert np.mean(r_beta > 1.1) < 0.01 and np.mean(r_gam > 1.1) < 0.01
    assert np.all(r_hyp < 1.2), r_hyp
    # the same factor from the traced draws of the traced genes
    tb = np.stack([t[:, 2 + 2 * L:].reshape(post, T, L + 1)[:, :, 1:] for t in traces])     # [C, M, T, L]
    r_tr = diagnostics.rhat_from_moments(tb.mean(1), (tb ** 2).mean(1), post)
    np.testing.assert_allclose(r_tr, r_beta[genes], rtol=1e-4)
