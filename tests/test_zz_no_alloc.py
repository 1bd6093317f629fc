"""gs_loss_image_noalloc (the entry point that allocates nothing) against
gs_loss_image, called through the C ABI: two calls in a row, the second on a
smaller stack, each bitwise equal to the plan-based call on the same inputs
(the two share their kernels, so the loss and the gradient are the same
numbers).  Sizes beyond the static buffer are refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2405_20693_amd import _native as N
from paper_2405_20693_amd import ops

pytestmark = pytest.mark.gpu


def _stack(seed, n, h, w):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (n, h, w)).astype(np.float32)
    y = np.clip(x + rng.normal(0.0, 0.1, (n, h, w)), 0.0, None).astype(np.float32)
    return torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()


def _noalloc(x, y, lam, grad):
    n, h, w = x.shape
    loss = torch.full((3,), float("nan"), device=x.device)
    g = torch.full_like(x, float("nan")) if grad else None
    st = N.lib().gs_loss_image_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       n, h, w, ctypes.c_float(lam),
                                       ctypes.c_void_p(loss.data_ptr()),
                                       ctypes.c_void_p(g.data_ptr()) if grad else None,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, N.lib().gs_last_error()
    return loss, g


def test_noalloc_loss_matches_plan_loss_on_two_calls():
    torch.cuda.set_device(0)
    plan = ops.Plan()
    # a stack for the marching loss kernel, then ragged stacks for the tile
    # kernel, each smaller than the one before: a call's partial sums overwrite
    # only part of what the earlier ones left in the shared buffer
    for seed, shape in ((2, (512, 65, 55)), (3, (5, 300, 277)), (4, (2, 45, 70))):
        x, y = _stack(seed, *shape)
        for grad in (True, False):
            ref_loss, ref_g = ops.image_loss(x, y, plan, 0.25, grad=grad)
            loss, g = _noalloc(x, y, 0.25, grad)
            torch.cuda.synchronize()
            print(f"noalloc {shape} grad={grad}: loss {loss.tolist()} vs {ref_loss.tolist()}",
                  flush=True)
            assert torch.equal(loss, ref_loss)
            if grad:
                assert torch.equal(g, ref_g)


def test_noalloc_loss_rejects_stacks_beyond_its_buffer():
    torch.cuda.set_device(0)
    x = torch.zeros(1, device="cuda")
    tiles_max = 262144
    n = tiles_max // 64 + 1  # 64 tiles of 32 x 32 per 256 x 256 image
    st = N.lib().gs_loss_image_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                       n, 256, 256, ctypes.c_float(0.25),
                                       ctypes.c_void_p(x.data_ptr()), None, None)
    assert st == 5 and b"static buffer" in N.lib().gs_last_error()
