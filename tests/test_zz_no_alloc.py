"""The allocation-free loss entry point against the one with a caller's workspace.

cnn_mse_grad_noalloc keeps its per-block partial sums in a fixed device array inside the
library; cnn_mse_grad writes them to a workspace the caller passes. Both go through the
C ABI. The gradient must be identical bit for bit (same kernel, same inputs) and the
loss must equal the workspace's partials summed in block order and divided by the
element count. Two calls in a row, the second with a smaller input, show that the array
keeps nothing from one call to the next that the result depends on.
"""
import sys

import numpy as np
import pytest

from paper_2607_01591_amd import cnn

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(shape, cv, seed, cuda):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    y = torch.randn(shape, generator=g, dtype=torch.float32).to(cuda)
    t = torch.randn(shape, generator=g, dtype=torch.float32).to(cuda)
    return y, t, cv


def test_noalloc_loss_matches_workspace_call(cuda):
    import torch
    # 8 images of 128 x 128 x 32 channels (7 used), then 2 images of 40 x 24 x 16 (5 used)
    for shape, cv, seed in [((8, 128, 128, 32), 7, 1), ((2, 40, 24, 16), 5, 2)]:
        log(f"[no-alloc loss] shape {shape}, {cv} channels used")
        y, t, cv = _case(shape, cv, seed, cuda)
        dy_ref = torch.empty_like(y)
        parts = torch.zeros(256, dtype=torch.float64, device=cuda)
        cnn.mse_grad(y, t, cv, dy_ref, parts)
        dy = torch.full_like(y, float("nan"))
        loss = torch.full((1,), float("nan"), dtype=torch.float64, device=cuda)
        cnn.mse_grad_noalloc(y, t, cv, dy, loss)
        torch.cuda.synchronize()
        assert torch.equal(dy, dy_ref)
        p = parts.cpu().numpy()
        inv_count = 1.0 / (float(y.numel() // shape[-1]) * float(cv))
        ref = 0.0
        for v in p:                     # block order, as the library sums them
            ref += float(v)
        ref *= inv_count
        got = float(loss.item())
        # independent check of the value itself (FP64 on the host)
        d = (y - t)[..., :cv].double().cpu().numpy()
        exact = float(np.mean(d * d))
        log(f"  loss {got:.15e}, from the workspace partials {ref:.15e}, host FP64 {exact:.15e}")
        assert got == ref
        assert abs(got - exact) <= 1e-12 * exact


def test_noalloc_rejects_bad_arguments(cuda):
    import torch
    y = torch.zeros((1, 4, 4, 8), dtype=torch.float32, device=cuda)
    loss = torch.zeros(1, dtype=torch.float64, device=cuda)
    with pytest.raises(Exception):
        cnn.mse_grad_noalloc(y, y, 9, torch.empty_like(y), loss)     # more used channels than stored
