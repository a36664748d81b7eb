"""The long-run chain comparisons have the right size and power (CPU only):
two oracle chains with different seeds agree; a chain from an oracle with a
planted mistake does not.  The plain sampler on the two-group design uses the
calibrated bar of agree(); the shift step with exact draws, on the two-group
design and at the Section 5 design (N = 16, L = 5), the within-3-MCSE bar of
agree_3mcse()."""
import os

import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.chain_compare import agree, agree_3mcse, compare

ITERS, BURNIN = 2000, 500


def oracle_draws(o, ds):
    post = ITERS - BURNIN
    o.sweep(BURNIN)
    hyp = np.empty((post, 2 + 2 * ds.L))
    gam = np.empty((post, ds.G))
    beta = np.empty((post, ds.G, ds.L))
    for i in range(post):
        o.sweep(1)
        st = o.get_state()
        hyp[i], gam[i], beta[i] = st["hyp"], st["gam"], st["beta"]
    o.close()
    return hyp, gam, beta


@pytest.mark.slow
def test_chain_comparison_size_and_power(oracle_lib):
    ds = datagen.small_two_group(G=1000, seed=0)
    threads = min(8, os.cpu_count() or 1)
    kw = dict(burnin=BURNIN, tune_start=BURNIN // 10, threads=threads)
    a = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=21, **kw), ds)
    b = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=22, **kw), ds)
    r = compare(*a, *b)
    assert agree(r), r
    c = oracle_draws(oracle_lib.variant(2).Oracle(ds.y, ds.X, ds.h, seed=22, **kw), ds)
    r2 = compare(*a, *c)
    assert not agree(r2), r2


@pytest.mark.slow
def test_within_3mcse_size_and_power(oracle_lib):
    threads = min(8, os.cpu_count() or 1)
    mask = 0xFE | (1 << 11) | (1 << 12)
    kw = dict(burnin=BURNIN, tune_start=BURNIN // 10, threads=threads, update_mask=mask)
    ds = datagen.small_two_group(G=1000, seed=0)
    a = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=41, **kw), ds)
    b = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=42, **kw), ds)
    r = compare(*a, *b)
    assert agree_3mcse(r), r
    ds = datagen.paper_design_16(G=2000, seed=0)
    a = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=41, **kw), ds)
    b = oracle_draws(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=42, **kw), ds)
    r = compare(*a, *b)
    assert agree_3mcse(r), r
    # planted mistakes: the beta statistic of the wrong column; the scale of
    # the exact gamma_g draw nu tau instead of nu tau / 2
    for mutant in (5, 15):
        c = oracle_draws(oracle_lib.variant(mutant).Oracle(ds.y, ds.X, ds.h, seed=42, **kw), ds)
        r2 = compare(*a, *c)
        assert not agree_3mcse(r2), (mutant, r2)
