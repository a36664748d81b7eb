"""The allocation-free entry point fb_mlp_loss_grad_noalloc against
fb_mlp_loss_grad, through the C ABI.

Both run the same kernels on the same inputs: the gradient blocks must be
identical bit for bit and the mean loss equal to FP32 rounding (its FP64 sum
runs in another order).  Two calls in a row, the second with fewer rows, so
the shared static scratch is reused with a smaller batch; then the rejected
sizes.
"""
import numpy as np
import pytest

from tests.gpu_common import require_gpu, say
from tests.test_oracle_mlp import random_model

pytestmark = pytest.mark.gpu


def _params(F, L, seed):
    from tests.test_gpu_mlp import to_gpu_params
    return to_gpu_params(random_model(np.random.default_rng(seed), L), L)


def _run_noalloc(F, torch, params, L, phi, tgt, stream):
    dev = torch.device("cuda:0")
    master = torch.from_numpy(F.mlp_master_block(params)).to(dev)
    d_phi = torch.from_numpy(np.ascontiguousarray(phi, np.float32)).to(dev)
    d_tgt = torch.from_numpy(np.ascontiguousarray(tgt, np.float32)).to(dev)
    loss = torch.full((1,), np.nan, dtype=torch.float32, device=dev)
    grad = torch.full((F.FB_MLP_PARAMS,), np.nan, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    F.fb_mlp_loss_grad_noalloc(master.data_ptr(), L, d_phi.data_ptr(), d_tgt.data_ptr(), phi.shape[0],
                               loss.data_ptr(), grad.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return float(loss.cpu().numpy()[0]), grad.cpu().numpy()


def test_noalloc_loss_grad_matches_the_allocating_entry_point():
    F = require_gpu()
    import torch
    stream = torch.cuda.Stream()
    for B, L, seed in ((512, 5, 11), (96, 3, 12)):
        say("noalloc case", "B", B, "L", L, "seed", seed)
        rng = np.random.default_rng(seed + 100)
        params = _params(F, L, seed)
        phi = rng.normal(0, 1.5, (B, 32)).astype(np.float32)
        tgt = rng.normal(0, 1, (B, L)).astype(np.float32)
        loss_ref, grads_ref = F.fb_mlp_loss_grad(params, L, phi, tgt)
        loss_na, grad_na = _run_noalloc(F, torch, params, L, phi, tgt, stream)
        ref = F.mlp_master_block(grads_ref)
        say("loss", loss_ref, loss_na, "max |grad diff|", float(np.max(np.abs(grad_na - ref))))
        assert np.isfinite(grad_na).all()
        assert np.array_equal(grad_na, ref)
        assert abs(loss_na - loss_ref) <= 1e-6 * abs(loss_ref), (loss_na, loss_ref)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    F = require_gpu()
    import torch
    dev = torch.device("cuda:0")
    L = 2
    big = F.FB_NOALLOC_MAX_ROWS + 32
    master = torch.zeros(F.FB_MLP_PARAMS, dtype=torch.float32, device=dev)
    phi = torch.zeros(big * 32, dtype=torch.float32, device=dev)
    tgt = torch.zeros(big * L, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = torch.zeros(F.FB_MLP_PARAMS, dtype=torch.float32, device=dev)
    ptrs = (master.data_ptr(), L, phi.data_ptr(), tgt.data_ptr())
    for B in (big, 48, 0):
        with pytest.raises(F.FbError) as ei:
            F.fb_mlp_loss_grad_noalloc(*ptrs, B, loss.data_ptr(), grad.data_ptr(), 0)
        assert ei.value.code == F.FB_EINVAL
    with pytest.raises(F.FbError):
        F.fb_mlp_loss_grad_noalloc(master.data_ptr(), 9, phi.data_ptr(), tgt.data_ptr(), 64, loss.data_ptr(),
                                   grad.data_ptr(), 0)
    # a weight block that is not 16-byte aligned is rejected on the host
    with pytest.raises(F.FbError) as ei:
        F.fb_mlp_loss_grad_noalloc(master.data_ptr() + 4, L, phi.data_ptr(), tgt.data_ptr(), 64, loss.data_ptr(),
                                   grad.data_ptr(), 0)
    assert ei.value.code == F.FB_EINVAL
    torch.cuda.synchronize()
