"""A context whose device memory comes from the caller's allocator
(fb_options.dev_alloc / dev_free), here PyTorch's caching allocator (GPU only).

The draws do not depend on where the arrays live: a context on PyTorch's
memory gives the same chain bit for bit as one on hipMalloc, the memory shows
up in PyTorch's accounting while the context lives and goes back to it at
destroy, and allocator failures become clean errors.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.gpu_common import STATE_KEYS, require_gpu, say

pytestmark = pytest.mark.gpu


def _run(F, ds, sweeps, **kw):
    s = F.Sampler(ds.y, ds.X, ds.h, seed=7, burnin=10, tune_start=2, precision=1, jitter=0, thin=1,
                  trace_genes=8, trace_capacity=sweeps, **kw)
    s.sweep(sweeps)
    assert s.sync() == 0
    st = F.fb_get_state(s.ctx)
    summ = F.fb_summaries(s.ctx)
    tr, _ = F.fb_trace(s.ctx)
    return s, st, summ, tr


def test_torch_memory_gives_the_same_chain():
    F = require_gpu()
    import torch
    ds = datagen.paper_design_16(G=3000, seed=2)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    s1, st1, sm1, tr1 = _run(F, ds, 25, torch_memory=True)
    held = torch.cuda.memory_allocated() - base
    say("context memory held by the caching allocator:", held, "bytes")
    # at least eps, its widths and its FP64 moments
    assert held >= ds.G * ds.N * (4 + 4 + 4 + 16)
    s2, st2, sm2, tr2 = _run(F, ds, 25)
    for k in STATE_KEYS:
        assert np.array_equal(st1[k], st2[k]), k
    for k in sm1:
        assert np.array_equal(np.asarray(sm1[k]), np.asarray(sm2[k])), k
    assert np.array_equal(tr1, tr2)
    # the autotuner's snapshot goes through the allocator too
    F.fb_autotune(s1.ctx, 2)
    s1.close()
    s2.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_allocator_failures_are_errors():
    F = require_gpu()
    import torch
    ds = datagen.small_two_group(G=200, seed=1)
    # an allocator that has no memory
    none_alloc = F.DEV_ALLOC_FN(lambda n, u: None)
    no_free = F.DEV_FREE_FN(lambda p, u: None)
    opts = F.fb_default_options(burnin=10, tune_start=2)
    opts.dev_alloc, opts.dev_free = none_alloc, no_free
    with pytest.raises(F.FbError) as ei:
        F.fb_create(ds.y, ds.X, ds.h, seed=1, options=opts)
    assert ei.value.code == F.FB_ENOMEM
    # one that returns memory off the 256-byte grid: rejected and given back
    held = {}

    def off_grid(n, u):
        p = torch.cuda.caching_allocator_alloc(int(n) + 256)
        held[p + 4] = p
        return p + 4

    def give_back(p, u):
        torch.cuda.caching_allocator_delete(held.pop(p))

    a, f = F.DEV_ALLOC_FN(off_grid), F.DEV_FREE_FN(give_back)
    opts.dev_alloc, opts.dev_free = a, f
    with pytest.raises(F.FbError) as ei:
        F.fb_create(ds.y, ds.X, ds.h, seed=1, options=opts)
    assert ei.value.code == F.FB_EINVAL
    assert not held
    torch.cuda.synchronize()


def test_training_gives_its_scratch_back():
    """fb_proposal_train's temporaries (moments, Adam state, minibatch buffers,
    loss sums) go back to the allocator when the call returns: training twice
    on a context on PyTorch's memory leaves the same amount allocated."""
    F = require_gpu()
    import torch
    ds = datagen.paper_design_16(G=2000, seed=3)
    s = F.Sampler(ds.y, ds.X, ds.h, seed=5, burnin=100, tune_start=10, precision=1, torch_memory=True)
    s.sweep(50)
    F.fb_proposal_collect(s.ctx, 40, every=2)
    opts = F.fb_default_train_opts(epochs=3)
    F.fb_proposal_train(s.ctx, opts)
    torch.cuda.synchronize()
    after_first = torch.cuda.memory_allocated()
    F.fb_proposal_train(s.ctx, opts)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == after_first
    s.close()
