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
from tests.chain_compare import agree, compare
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
