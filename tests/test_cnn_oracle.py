"""Pins for the numpy CNN oracle: central finite differences of the loss, a 1x1
special case against a plain matrix product, shifted taps, and for dilated
convolutions the polyphase identity; the input features' spectrum in closed form for
two groups without up-scatter and one group."""
import numpy as np

from oracle import cnn_oracle as C


def _params(rng, chans):
    return [(rng.normal(0, 0.4, size=(co, 3, 3, ci)), rng.normal(0, 0.1, size=co))
            for ci, co in zip(chans[:-1], chans[1:])]


def test_conv_center_tap_is_matmul():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 4, 3))
    W = np.zeros((6, 3, 3, 3))
    W[:, 1, 1, :] = rng.normal(size=(6, 3))
    b = rng.normal(size=6)
    np.testing.assert_allclose(C.conv_forward(x, W, b), x @ W[:, 1, 1, :].T + b, rtol=1e-14)


def test_conv_shift_tap_and_zero_padding():
    x = np.zeros((1, 4, 4, 1))
    x[0, 2, 1, 0] = 1.0
    W = np.zeros((1, 3, 3, 1))
    W[0, 0, 2, 0] = 1.0            # z[y, x] = x[y - 1, x + 1]
    z = C.conv_forward(x, W, np.zeros(1))
    expect = np.zeros((1, 4, 4, 1))
    expect[0, 3, 0, 0] = 1.0
    np.testing.assert_array_equal(z, expect)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    params = _params(rng, [3, 5, 4, 2])
    x = rng.normal(size=(2, 6, 5, 3))
    t = rng.normal(size=(2, 6, 5, 2))
    y, acts, pre = C.forward(x, params)
    grads = C.backward(params, acts, pre, t)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = C.mse(C.forward(x, params)[0], t)
                flat[idx] = old - h
                lm = C.mse(C.forward(x, params)[0], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gf[idx]) < 1e-7 + 1e-5 * abs(fd), (li, idx, fd, gf[idx])


def test_input_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    W = rng.normal(size=(4, 3, 3, 3))
    x = rng.normal(size=(1, 5, 5, 3))
    dz = rng.normal(size=(1, 5, 5, 4))
    dx, _, _ = C.conv_backward(x, W, dz)
    h = 1e-6
    for idx in rng.choice(x.size, size=15, replace=False):
        xf = x.reshape(-1)
        old = xf[idx]
        xf[idx] = old + h
        lp = np.sum(C.conv_forward(x, W, np.zeros(4)) * dz)
        xf[idx] = old - h
        lm = np.sum(C.conv_forward(x, W, np.zeros(4)) * dz)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - dx.reshape(-1)[idx]) < 1e-6


def test_adam_first_step_moves_by_lr():
    p, m, v = C.adam_step(np.array([1.0, -2.0]), np.array([0.3, -5.0]), np.zeros(2), np.zeros(2), 1, lr=0.01)
    np.testing.assert_allclose(p, [0.99, -1.99], rtol=1e-6)


def test_dilated_conv_acts_on_interleaved_sub_images():
    """Polyphase identity: with dilation d, output pixel (y, x) only sees inputs at
    (y + (ky-1) d, x + (kx-1) d), i.e. the sub-image of pixels congruent to (y, x) mod d,
    on which it is the plain 3x3 convolution."""
    rng = np.random.default_rng(4)
    W = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=3)
    for d in (2, 3):
        x = rng.normal(size=(2, 11, 9, 2))
        z = C.conv_forward(x, W, b, d)
        for a in range(d):
            for c in range(d):
                np.testing.assert_allclose(z[:, a::d, c::d, :], C.conv_forward(x[:, a::d, c::d, :], W, b),
                                           rtol=1e-13, atol=1e-13)


def test_dilated_shift_tap():
    x = np.zeros((1, 9, 9, 1))
    x[0, 2, 5, 0] = 1.0
    W = np.zeros((1, 3, 3, 1))
    W[0, 0, 2, 0] = 1.0            # z[y, x] = x[y - 3, x + 3] at d = 3
    z = C.conv_forward(x, W, np.zeros(1), 3)
    expect = np.zeros((1, 9, 9, 1))
    expect[0, 5, 2, 0] = 1.0
    np.testing.assert_array_equal(z, expect)


def test_dilated_gradients_match_central_differences():
    rng = np.random.default_rng(5)
    params = _params(rng, [2, 3, 2])
    dils = [2, 3]
    x = rng.normal(size=(1, 8, 7, 2))
    t = rng.normal(size=(1, 8, 7, 2))
    y, acts, pre = C.forward(x, params, dils)
    grads = C.backward(params, acts, pre, t, dils)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(10, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = C.mse(C.forward(x, params, dils)[0], t)
                flat[idx] = old - h
                lm = C.mse(C.forward(x, params, dils)[0], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gf[idx]) < 1e-7 + 1e-5 * abs(fd), (li, idx, fd, gf[idx])
    W = params[0][0]
    dz = rng.normal(size=(1, 8, 7, 3))
    dx, _, _ = C.conv_backward(x, W, dz, 2)
    for idx in rng.choice(x.size, size=12, replace=False):
        xf = x.reshape(-1)
        old = xf[idx]
        xf[idx] = old + h
        lp = np.sum(C.conv_forward(x, W, np.zeros(3), 2) * dz)
        xf[idx] = old - h
        lm = np.sum(C.conv_forward(x, W, np.zeros(3), 2) * dz)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - dx.reshape(-1)[idx]) < 1e-6


def test_material_features_closed_forms():
    """Two groups, no up-scatter: the spectrum is phi_1 = chi_1 / (St_1 - S_11),
    phi_2 = (chi_2 + S_12 phi_1) / (St_2 - S_22) in closed form; one group: phi = 1 (log
    0); a non-fissile material takes the mean fission spectrum of the fissile ones;
    Sigma_a is Sigma_t minus the scattering out of the group (not into it)."""
    st = np.array([[0.5, 1.2], [0.4, 0.9]])
    ss = np.array([[[0.30, 0.15], [0.0, 1.0]], [[0.35, 0.04], [0.0, 0.85]]])
    nsf = np.array([[0.01, 0.2], [0.0, 0.0]])
    chi = np.array([[0.9, 0.1], [0.0, 0.0]])
    f = C.material_features(st, ss, nsf, chi)
    for m, c in ((0, chi[0]), (1, chi[0])):          # material 1 takes material 0's chi
        p1 = c[0] / (st[m, 0] - ss[m, 0, 0])
        p2 = (c[1] + ss[m, 0, 1] * p1) / (st[m, 1] - ss[m, 1, 1])
        tot = p1 + p2
        np.testing.assert_allclose(f[m, :2], np.log([p1 / tot, p2 / tot]), rtol=1e-13)
        np.testing.assert_allclose(f[m, 2:4], st[m])
        np.testing.assert_allclose(f[m, 4:6], [st[m, 0] - ss[m, 0, 0] - ss[m, 0, 1], st[m, 1] - ss[m, 1, 1]])
        np.testing.assert_allclose(f[m, 6:], nsf[m])
    one = C.material_features([[1.0]], [[[0.6]]], [[0.3]], [[1.0]])
    np.testing.assert_allclose(one, [[0.0, 1.0, 0.4, 0.3]])
    # no fissile material at all: a flat source
    flat = C.material_features([[1.0, 2.0]], [[[0.5, 0.0], [0.0, 1.0]]], [[0.0, 0.0]], [[0.0, 0.0]])
    p = np.array([0.5 / 0.5, 0.5 / 1.0])
    np.testing.assert_allclose(flat[0, :2], np.log(p / p.sum()), rtol=1e-13)
