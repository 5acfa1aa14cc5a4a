"""Pins of the learned-guess oracle against facts that do not come from it:
brute-force loops on tiny grids, the convolution theorem, adjointness,
central differences of the loss, hand-computed Adam steps and circular
translation equivariance."""
import numpy as np
import pytest

from oracle import cnn_oracle as C


def brute_conv(x, w, b):
    """Direct loops over every output point, tap and channel."""
    H, W, cin = x.shape
    cout = w.shape[2]
    y = np.zeros((H, W, cout))
    for i in range(H):
        for j in range(W):
            for co in range(cout):
                acc = b[co]
                for ky in range(3):
                    for kx in range(3):
                        for ci in range(cin):
                            acc += w[ky, kx, co, ci] * x[(i + ky - 1) % H, (j + kx - 1) % W, ci]
                y[i, j, co] = acc
    return y


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(5, 7, 3))
    w = rng.normal(size=(3, 3, 4, 3))
    b = rng.normal(size=4)
    np.testing.assert_allclose(C.conv3x3(x, w, b), brute_conv(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv_delta_kernels_are_shifts():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(6, 8, 2))
    # centre tap, identity channel map: the identity
    w = np.zeros((3, 3, 2, 2))
    w[1, 1] = np.eye(2)
    np.testing.assert_array_equal(C.conv3x3(x, w), x)
    # tap (ky, kx) = (0, 2) reads x at (y - 1, x + 1)
    w = np.zeros((3, 3, 2, 2))
    w[0, 2] = np.eye(2)
    y = C.conv3x3(x, w)
    assert y[3, 4, 1] == x[2, 5, 1] and y[0, 7, 0] == x[5, 0, 0]


def test_conv_is_circular_correlation_by_fft():
    """One channel: y = IFFT(FFT(x) * conj(FFT(k))) with the 3x3 kernel placed
    around the origin of an H x W array (convolution theorem for correlation)."""
    rng = np.random.default_rng(2)
    H, W = 16, 12
    x = rng.normal(size=(H, W, 1))
    w = rng.normal(size=(3, 3, 1, 1))
    k = np.zeros((H, W))
    for ky in range(3):
        for kx in range(3):
            k[(ky - 1) % H, (kx - 1) % W] = w[ky, kx, 0, 0]
    ref = np.real(np.fft.ifft2(np.fft.fft2(x[..., 0]) * np.conj(np.fft.fft2(k))))
    np.testing.assert_allclose(C.conv3x3(x, w)[..., 0], ref, atol=1e-12)


def test_input_grad_is_the_adjoint():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(9, 6, 5))
    z = rng.normal(size=(9, 6, 4))
    w = rng.normal(size=(3, 3, 4, 5))
    lhs = np.sum(C.conv3x3(x, w) * z)
    rhs = np.sum(x * C.conv3x3_input_grad(z, w))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_network_gradients_match_central_differences():
    rng = np.random.default_rng(4)
    net = C.init_net(rng, cin=3, ch=4, layers=3, cout=1)
    for b in net.b:
        b += rng.normal(scale=0.1, size=b.shape)
    x = rng.normal(size=(6, 5, 3))
    target = rng.normal(size=(6, 5))
    loss, gw, gb = C.backward(net, C.forward(net, x), target)
    eps = 1e-6
    picks = [(0, (0, 1, 2, 1)), (1, (2, 2, 3, 0)), (2, (1, 0, 0, 3)), (1, (1, 1, 1, 1))]
    for l, idx in picks:
        orig = net.w[l][idx]
        net.w[l][idx] = orig + eps
        lp = C.mse(C.forward(net, x)[-1][..., 0], target)
        net.w[l][idx] = orig - eps
        lm = C.mse(C.forward(net, x)[-1][..., 0], target)
        net.w[l][idx] = orig
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gw[l][idx]) < 1e-6 * max(1.0, abs(fd)), (l, idx, fd, gw[l][idx])
    for l, co in [(0, 2), (2, 0)]:
        orig = net.b[l][co]
        net.b[l][co] = orig + eps
        lp = C.mse(C.forward(net, x)[-1][..., 0], target)
        net.b[l][co] = orig - eps
        lm = C.mse(C.forward(net, x)[-1][..., 0], target)
        net.b[l][co] = orig
        assert abs((lp - lm) / (2 * eps) - gb[l][co]) < 1e-6


def test_adam_two_scalar_steps_by_hand():
    """p = 1, g = 0.5 then g = -0.25, lr = 0.1, beta1 = 0.9, beta2 = 0.999, eps = 0:
    step 1: m = 0.05, v = 0.00025, mhat = 0.5, vhat = 0.25 -> p = 1 - 0.1 = 0.9;
    step 2: m = 0.045 - 0.025 = 0.02, v = 0.00024975 + 0.0000625 = 0.00031225,
    mhat = 0.02 / 0.19 = 0.105263..., vhat = 0.00031225 / 0.001999 = 0.156203...,
    p = 0.9 - 0.1 * 0.105263 / 0.395225 = 0.873366..."""
    opt = C.Adam(lr=0.1, eps=0.0)
    p = [np.array([1.0])]
    C.adam_step(opt, p, [np.array([0.5])])
    assert abs(p[0][0] - 0.9) < 1e-15
    C.adam_step(opt, p, [np.array([-0.25])])
    mhat = 0.02 / (1 - 0.9 ** 2)
    vhat = (0.999 * 0.00025 + 0.001 * 0.0625) / (1 - 0.999 ** 2)
    assert abs(p[0][0] - (0.9 - 0.1 * mhat / np.sqrt(vhat))) < 1e-14
    assert abs(p[0][0] - 0.873366) < 1e-6


def test_network_is_translation_equivariant():
    rng = np.random.default_rng(5)
    net = C.init_net(rng, cin=3, ch=4, layers=4, cout=1)
    x = rng.normal(size=(8, 10, 3))
    y = C.forward(net, x)[-1]
    ys = C.forward(net, np.roll(x, (3, -4), axis=(0, 1)))[-1]
    np.testing.assert_allclose(ys, np.roll(y, (3, -4), axis=(0, 1)), atol=1e-12)


def test_features_scale_out():
    """The guess is linear in (r0, sigma_prev) for fixed h: doubling r0 doubles the correction."""
    rng = np.random.default_rng(6)
    net = C.init_net(rng, cin=3, ch=4, layers=3, cout=1)
    r0, mr, h = rng.normal(size=(6, 6)), rng.normal(size=(6, 6)), 1 + 0.1 * rng.normal(size=(6, 6))
    sp = rng.normal(size=(6, 6))
    g1 = C.guess(net, sp, r0, mr, h) - sp
    g2 = C.guess(net, sp, 2 * r0, 2 * mr, h) - sp
    np.testing.assert_allclose(g2, 2 * g1, atol=1e-12)
    x, s = C.features(r0, mr, h)
    assert abs(C.rms(x[..., 0]) - 1.0) < 1e-12 and s > 0


def backward_without_relu_mask(net, acts, target):
    """A plausible slip: the gradient passed through the ReLUs unmasked."""
    n = len(net.w)
    pred = acts[-1][..., 0]
    d = np.zeros_like(acts[-1])
    d[..., 0] = 2.0 * (pred - target) / pred.size
    gw = [None] * n
    for l in range(n - 1, -1, -1):
        gw[l], _ = C.conv3x3_weight_grad(d, acts[l])
        if l > 0:
            d = C.conv3x3_input_grad(d, net.w[l])
    return gw


@pytest.mark.parametrize("mistake", ["flip_tap", "drop_relu_mask", "transpose_taps"])
def test_planted_mistakes_fail_a_pin(mistake, monkeypatch):
    """Each plausible slip in the oracle breaks at least one pin above."""
    rng = np.random.default_rng(7)
    if mistake == "flip_tap":
        orig = C.conv3x3
        monkeypatch.setattr(C, "conv3x3", lambda x, w, b=None: orig(x, w[::-1, ::-1], b))
        x = rng.normal(size=(5, 7, 3)); w = rng.normal(size=(3, 3, 4, 3)); b = rng.normal(size=4)
        assert not np.allclose(C.conv3x3(x, w, b), brute_conv(x, w, b))
    elif mistake == "drop_relu_mask":
        net = C.init_net(rng, cin=3, ch=4, layers=3, cout=1)
        x = rng.normal(size=(6, 5, 3)); t = rng.normal(size=(6, 5))
        gw = backward_without_relu_mask(net, C.forward(net, x), t)
        eps, l, idx = 1e-6, 0, (1, 1, 2, 1)
        orig = net.w[l][idx]
        net.w[l][idx] = orig + eps
        lp = C.mse(C.forward(net, x)[-1][..., 0], t)
        net.w[l][idx] = orig - eps
        lm = C.mse(C.forward(net, x)[-1][..., 0], t)
        assert abs((lp - lm) / (2 * eps) - gw[l][idx]) > 1e-4
    else:
        x = rng.normal(size=(9, 6, 5)); z = rng.normal(size=(9, 6, 4)); w = rng.normal(size=(3, 3, 4, 5))
        lhs = np.sum(C.conv3x3(x, w) * z)
        wt = np.transpose(w, (1, 0, 2, 3))  # ky and kx exchanged
        rhs = np.sum(x * C.conv3x3_input_grad(z, wt))
        assert abs(lhs - rhs) > 1e-6 * abs(lhs)
