"""GPU checks of the BF16 matrix-core network kernels against the FP64 numpy oracle.

Single kernels run on BF16-representable inputs, so the only differences are FP32
accumulation order (tolerance 1e-5 relative). The whole network's gradients are
compared at BF16 level (relative L2 error <= 3e-2), since activations are rounded to
BF16 between layers.
"""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as CO

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bf(a, cuda):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device=cuda).to(torch.bfloat16)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("N,H,W,Ci,Co,relu,d", [(2, 5, 70, 32, 16, False, 1), (1, 4, 64, 64, 64, True, 1),
                                                 (1, 3, 20, 32, 32, True, 1), (2, 9, 70, 32, 32, True, 2),
                                                 (1, 12, 40, 64, 64, False, 4), (1, 5, 20, 32, 16, False, 16),
                                                 (1, 3, 130, 32, 64, True, 2), (2, 4, 128, 64, 32, False, 1),
                                                 (1, 2, 200, 32, 16, False, 8)])
def test_conv_forward_exact(N, H, W, Ci, Co, relu, d, cuda):
    import torch
    from paper_2607_01591_amd import cnn
    log(f"[cnn fwd] {N}x{H}x{W} {Ci}->{Co} dilation {d}")
    rng = np.random.default_rng(0)
    x = _bf(rng.normal(size=(N, H, W, Ci)), cuda)
    w = _bf(rng.normal(0, 0.2, size=(Co, 9, Ci)), cuda)
    b = torch.as_tensor(rng.normal(size=Co).astype(np.float32), device=cuda)
    yf = torch.empty((N, H, W, Co), dtype=torch.float32, device=cuda)
    yb = torch.empty((N, H, W, Co), dtype=torch.bfloat16, device=cuda)
    cnn.conv3x3(x, w, b, relu=relu, out_bf16=yb, out_f32=yf, dilation=d)
    ref = CO.conv_forward(_np(x), _np(w).reshape(Co, 3, 3, Ci), _np(b), d)
    if relu:
        ref = np.maximum(ref, 0)
    np.testing.assert_allclose(_np(yf), ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())
    np.testing.assert_allclose(_np(yb), ref, rtol=1e-2, atol=1e-2 * np.abs(ref).max())


@pytest.mark.parametrize("d", [1, 3, 8])
def test_wgrad_and_dgrad_exact(d, cuda):
    import torch
    from paper_2607_01591_amd import cnn
    log(f"[cnn wgrad/dgrad] dilation {d}")
    rng = np.random.default_rng(1)
    N, H, W, Ci, Co = 2, 10, 40, 32, 32
    x = _bf(rng.normal(size=(N, H, W, Ci)), cuda)
    dz = _bf(rng.normal(size=(N, H, W, Co)), cuda)
    w = rng.normal(0, 0.2, size=(Co, 9, Ci)).astype(np.float32)
    w_bf = _np(_bf(w, cuda))                       # the dgrad kernel rounds weights to BF16
    dx_ref, dW_ref, _ = CO.conv_backward(_np(x), w_bf.reshape(Co, 3, 3, Ci), _np(dz), d)
    dW = torch.zeros((Co, 9, Ci), dtype=torch.float32, device=cuda)
    cnn.wgrad(x, dz, dW, dilation=d)
    np.testing.assert_allclose(_np(dW), dW_ref.reshape(Co, 9, Ci), rtol=1e-5, atol=1e-5 * np.abs(dW_ref).max())
    wt = torch.empty((Ci, 9, Co), dtype=torch.bfloat16, device=cuda)
    cnn.weights_for_dgrad(torch.as_tensor(w, device=cuda), wt)
    dx = torch.empty((N, H, W, Ci), dtype=torch.float32, device=cuda)
    cnn.conv3x3(dz, wt, None, relu=False, out_f32=dx, dilation=d)
    np.testing.assert_allclose(_np(dx), dx_ref, rtol=1e-5, atol=1e-5 * np.abs(dx_ref).max())


@pytest.mark.parametrize("N,H,W,Ci,Co,d", [(1, 6, 128, 64, 64, 1), (1, 5, 200, 64, 32, 3), (2, 4, 70, 32, 64, 2),
                                            (1, 40, 33, 64, 16, 32), (1, 9, 131, 32, 32, 8), (1, 3, 20, 96, 32, 1),
                                            (1, 4, 16, 32, 48, 1)])
def test_wgrad_shapes(N, H, W, Ci, Co, d, cuda):
    """Weight gradient against the oracle over the staged kernel's cases (one and several
    128-pixel segments with a ragged last one, shifts at every alignment, dilation 32 with
    rows whose x row leaves the image) and two shapes it hands to the gather kernel
    (Ci = 96, Co = 48). dW is accumulated into a non-zero start."""
    import torch
    from paper_2607_01591_amd import cnn
    log(f"[cnn wgrad] {N}x{H}x{W} {Ci}->{Co} dilation {d}")
    rng = np.random.default_rng(7)
    x = _bf(rng.normal(size=(N, H, W, Ci)), cuda)
    dz = _bf(rng.normal(size=(N, H, W, Co)), cuda)
    w0 = rng.normal(size=(Co, 9, Ci)).astype(np.float32)
    _, dW_ref, _ = CO.conv_backward(_np(x), np.zeros((Co, 3, 3, Ci)), _np(dz), d)
    dW = torch.as_tensor(w0, device=cuda)
    cnn.wgrad(x, dz, dW, dilation=d)
    ref = dW_ref.reshape(Co, 9, Ci) + w0
    np.testing.assert_allclose(_np(dW), ref, rtol=1e-5, atol=1e-5 * np.abs(dW_ref).max())


@pytest.mark.parametrize("npix,Co", [(1000, 16), (70001, 64), (513, 48), (300, 512)])
def test_bias_grad(npix, Co, cuda):
    """db += column sums of FP32 dz: the coalesced kernel (Co dividing 256) and the
    per-channel one (Co = 48, 512)."""
    import torch
    from paper_2607_01591_amd import cnn
    rng = np.random.default_rng(3)
    dz = rng.normal(size=(npix, Co)).astype(np.float32)
    db0 = rng.normal(size=Co).astype(np.float32)
    db = torch.as_tensor(db0, device=cuda)
    cnn.bias_grad(torch.as_tensor(dz, device=cuda), db)
    ref = dz.astype(np.float64).sum(axis=0) + db0
    np.testing.assert_allclose(_np(db), ref, rtol=1e-5, atol=1e-5 * np.sqrt(npix))


@pytest.mark.parametrize("dils", [[1, 1, 1], [1, 4, 2]])
def test_network_gradients_match_oracle(dils, cuda):
    import torch
    from paper_2607_01591_amd import cnn
    log(f"[cnn network gradients] dilations {dils}")
    rng = np.random.default_rng(2)
    chans = [32, 32, 32, 32]
    net = cnn.ConvNet(chans, cuda, seed=3, in_used=32, out_used=5, dilations=dils)
    N, H, W = 2, 8, 64
    x = _bf(rng.normal(size=(N, H, W, 32)), cuda)
    t = torch.as_tensor(rng.normal(size=(N, H, W, 32)).astype(np.float32), device=cuda)
    loss, grads = net.gradients(x, t, cv=5)
    params = [(_np(net.Wb[i]).reshape(co, 3, 3, ci), _np(net.b[i])) for i, (ci, co) in
              enumerate(zip(chans[:-1], chans[1:]))]
    y, acts, pre = CO.forward(_np(x), params, dils)
    tt = _np(t).copy()
    tt[..., 5:] = y[..., 5:]                   # padding channels carry no loss
    ref = CO.backward(params, acts, pre, tt, dils)
    scale = y[..., :5].size / y.size           # oracle MSE averages over all channels
    loss_ref = np.mean((y[..., :5] - _np(t)[..., :5]) ** 2)
    assert abs(loss - loss_ref) < 2e-2 * loss_ref
    for li in range(len(chans) - 1):
        for g_gpu, g_ref in ((grads[li][0], ref[li][0]), (grads[li][1], ref[li][1])):
            a = _np(g_gpu).reshape(-1)
            b = (g_ref / scale).reshape(-1)
            err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            assert err < 3e-2, (li, err)


def test_adam_matches_oracle(cuda):
    import torch
    from paper_2607_01591_amd import cnn
    rng = np.random.default_rng(4)
    p0, g = rng.normal(size=1000), rng.normal(size=1000)
    p = torch.as_tensor(p0.astype(np.float32), device=cuda)
    gt = torch.as_tensor(g.astype(np.float32), device=cuda)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    pr, mr, vr = p0.copy(), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        cnn.adam(p, gt, m, v, step, lr=1e-2)
        pr, mr, vr = CO.adam_step(pr, g, mr, vr, step, lr=1e-2)
    np.testing.assert_allclose(_np(p), pr, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(cuda):
    import torch
    from paper_2607_01591_amd import cnn
    log("[cnn training]")
    rng = np.random.default_rng(5)
    N, H, W = 4, 16, 64
    xin = rng.normal(size=(N, H, W, 32)).astype(np.float32)
    # target: a fixed smooth function of the inputs (a blurred linear map)
    tgt = np.zeros((N, H, W, 32), np.float32)
    tgt[..., :3] = xin[..., :3] * 0.5 + 0.25 * np.roll(xin[..., 3:6], 1, axis=2)
    net = cnn.ConvNet([32, 32, 32, 32], cuda, seed=1, out_used=3)
    x = _bf(xin, cuda)
    t = torch.as_tensor(tgt, device=cuda)
    losses = [net.train_step(x, t, cv=3, lr=3e-3) for _ in range(60)]
    assert losses[-1] < 0.3 * losses[0], (losses[0], losses[-1])


def test_gather_and_bilinear(cuda):
    import torch
    from paper_2607_01591_amd import cnn
    rng = np.random.default_rng(6)
    table = rng.normal(size=(5, 3)).astype(np.float32)
    idx = rng.integers(0, 5, size=(4, 6)).astype(np.int32)
    out = torch.empty((4, 6, 8), dtype=torch.bfloat16, device=cuda)
    cnn.gather_rows(torch.as_tensor(table, device=cuda), torch.as_tensor(idx, device=cuda), 8, out)
    ref = np.zeros((4, 6, 8))
    ref[..., :3] = table[idx]
    np.testing.assert_allclose(_np(out), ref, rtol=1e-2, atol=1e-2)
    img = rng.normal(size=(4, 6, 8)).astype(np.float32)
    uv = np.array([[0.0, 0.0], [2.5, 1.25], [5.0, 3.0], [-1.0, 7.0]], np.float32)
    o = torch.empty((4, 3), dtype=torch.float64, device=cuda)
    cnn.bilinear(torch.as_tensor(img, device=cuda), 3, torch.as_tensor(uv, device=cuda), o, apply_exp=False)
    def bil(u, v):
        u, v = min(max(u, 0), 5), min(max(v, 0), 3)
        x0, y0 = min(int(u), 4), min(int(v), 2)
        fx, fy = u - x0, v - y0
        return ((1 - fy) * ((1 - fx) * img[y0, x0] + fx * img[y0, x0 + 1])
                + fy * ((1 - fx) * img[y0 + 1, x0] + fx * img[y0 + 1, x0 + 1]))[:3]
    np.testing.assert_allclose(o.cpu().numpy(), np.array([bil(*p) for p in uv]), rtol=1e-6, atol=1e-6)


def test_center_matches_numpy(cuda):
    """cnn_center: per image, the mean over pixels and used channels is removed from
    those entries; padded channels are left alone."""
    import torch
    from paper_2607_01591_amd import cnn
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3, 20, 17, 8)).astype(np.float32)
    t = torch.as_tensor(x, device=cuda)
    cnn.center(t, 7)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    ref = x.astype(np.float64)
    ref[..., :7] -= ref[..., :7].reshape(3, -1).mean(axis=1)[:, None, None, None]
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6)


def test_d4_transforms(cuda):
    """The 8 square symmetries: op 0 identity, 1-3 rotations, 4 transpose, 5 and 7
    mirrors, 6 anti-transpose; every op is a permutation, the 8 are distinct, op 2 is
    the 180-degree rotation, op 1 composed with itself is op 2, and transforming then
    accumulating with the same op gives back the image."""
    import torch
    from paper_2607_01591_amd import cnn
    rng = np.random.default_rng(8)
    S, Cc = 12, 32
    x = rng.normal(size=(1, S, S, Cc)).astype(np.float32)
    xb = _bf(x, cuda)
    xr = _np(xb)[0]
    outs = []
    for op in range(8):
        y = torch.empty_like(xb)
        cnn.d4_transform(xb, op, y)
        outs.append(_np(y)[0])
    np.testing.assert_array_equal(outs[0], xr)
    np.testing.assert_array_equal(outs[4], xr.transpose(1, 0, 2))
    np.testing.assert_array_equal(outs[5], xr[:, ::-1])
    np.testing.assert_array_equal(outs[7], xr[::-1, :])
    np.testing.assert_array_equal(outs[2], xr[::-1, ::-1])
    np.testing.assert_array_equal(outs[6], xr[::-1, ::-1].transpose(1, 0, 2))
    keys = {o.tobytes() for o in outs}
    assert len(keys) == 8
    for o in outs:
        np.testing.assert_array_equal(np.sort(o.ravel()), np.sort(xr.ravel()))
    y1 = torch.empty_like(xb)
    cnn.d4_transform(xb, 1, y1)
    y11 = torch.empty_like(xb)
    cnn.d4_transform(y1, 1, y11)
    np.testing.assert_array_equal(_np(y11)[0], outs[2])
    for op in range(8):
        y = torch.empty_like(xb)
        cnn.d4_transform(xb, op, y)
        acc = torch.zeros((S, S, Cc), dtype=torch.float32, device=cuda)
        cnn.d4_accumulate(y[0].float().contiguous(), Cc, op, 1.0, acc)
        np.testing.assert_array_equal(_np(acc), xr)


def test_material_features_match_oracle(cuda):
    """The feature kernel against the oracle's numpy solve: the 7-group lattice family's
    materials (fissile and not), random 2- and 12-group materials with up-scatter, and a
    set with no fissile material."""
    import torch
    from paper_2607_01591_amd import cnn
    from paper_2607_01591_amd import problems as P
    rng = np.random.default_rng(11)
    cases = []
    p = P.config(5, seed=200004)
    cases.append((p.sigma_t, p.sigma_s, p.nu_sigma_f, p.chi))
    for G in (2, 12):
        M = 5
        st = rng.uniform(0.3, 2.0, size=(M, G))
        ss = rng.uniform(0.0, 1.0, size=(M, G, G)) * (0.8 * st[:, :, None] / G)
        nsf = rng.uniform(0.0, 0.3, size=(M, G)) * (rng.uniform(size=(M, 1)) < 0.6)
        chi = rng.uniform(size=(M, G))
        chi /= chi.sum(axis=1, keepdims=True)
        cases.append((st, ss, nsf, chi))
    cases.append((cases[1][0], cases[1][1], np.zeros_like(cases[1][2]), cases[1][3]))
    for st, ss, nsf, chi in cases:
        M, G = st.shape
        dev = [torch.as_tensor(np.ascontiguousarray(a, np.float64), device=cuda) for a in (st, ss, nsf, chi)]
        out = torch.empty((M, 4 * G), dtype=torch.float32, device=cuda)
        cnn.material_features(*dev, out)
        ref = CO.material_features(st, ss, nsf, chi).astype(np.float32)
        np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
