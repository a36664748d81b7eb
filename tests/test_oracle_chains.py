"""The long-run chain comparison has the right size and power (CPU only): two
oracle chains with different seeds agree; a chain from an oracle with a
planted mistake (the gamma shape nu/2 + N instead of nu/2 + N/2) does not."""
import os

import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.chain_compare import agree, compare

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
