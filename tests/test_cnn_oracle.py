"""Pins of the FP64 network oracle (oracle/cnn_ref.py).

The convolution is checked against an explicit six-fold loop; every backward
operation against its adjoint identity <A x, y> = <x, A^T y> (exact up to
rounding, so a transposed index or a wrong sign shows); the whole network
gradient against central finite differences of its own loss.
"""
import numpy as np
import pytest

from oracle import cnn_ref as C


def test_conv_matches_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = C.conv3x3(x, w, b)
    B, H, W, _ = x.shape
    ref = np.zeros((B, H, W, 4))
    for bb in range(B):
        for i in range(H):
            for j in range(W):
                for o in range(4):
                    s = b[o]
                    for c in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                s += w[o, c, ky, kx] * x[bb, (i + ky - 1) % H, (j + kx - 1) % W, c]
                    ref[bb, i, j, o] = s
    assert np.abs(y - ref).max() < 1e-12


def test_conv_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 8, 5))
    w = rng.standard_normal((7, 5, 3, 3))
    gy = rng.standard_normal((2, 6, 8, 7))
    lhs = np.sum(C.conv3x3(x, w) * gy)
    assert abs(lhs - np.sum(x * C.conv3x3_data_grad(gy, w))) < 1e-10 * abs(lhs)
    gw, gb = C.conv3x3_weight_grad(x, gy)
    assert abs(lhs - np.sum(w * gw)) < 1e-10 * abs(lhs)
    assert np.allclose(gb, gy.sum(axis=(0, 1, 2)))


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 12, 3))
    y = rng.standard_normal((2, 4, 6, 3))
    assert abs(np.sum(C.pool2(x) * y) - np.sum(x * C.pool2_grad(y))) < 1e-12
    z = rng.standard_normal((2, 16, 24, 3))
    assert abs(np.sum(C.up2(x) * z) - np.sum(x * C.up2_grad(z))) < 1e-11


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.140625, 1e-3])
    r = C.round_bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0               # tie -> even
    assert r[2] == 1.0 + 2 ** -7     # tie -> even (upwards)
    assert r[3] == -3.140625
    assert abs(r[4] - 1e-3) / 1e-3 < 2 ** -8


@pytest.mark.parametrize("bf16", [False])
def test_network_gradient_finite_differences(bf16):
    rng = np.random.default_rng(3)
    n = C.num_params()
    params = np.zeros(n)
    o = 0
    for ci, co, _ in C.SPEC:
        params[o:o + co * ci * 9] = rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci))
        o += co * ci * 9
        params[o:o + co] = 0.05 * rng.standard_normal(co)
        o += co
    x = rng.standard_normal((2, 8, 8, 8))
    target = rng.standard_normal((2, 8, 8, 4))
    mask = rng.random((2, 8, 8)) > 0.2
    loss, g, _ = C.loss_and_grads(params, x, target, mask)
    idx = rng.choice(n, size=40, replace=False)
    # include the first and last layers' weights and a bias
    idx = np.concatenate([idx, [0, n - 1, n - 4, 8 * 32 * 9 + 1]])
    h = 1e-6
    for i in idx:
        p = params.copy()
        p[i] += h
        lp = C.loss_and_grads(p, x, target, mask)[0]
        p[i] -= 2 * h
        lm = C.loss_and_grads(p, x, target, mask)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])


# ------------------------------------------------------------------ Adam --
def test_adam_first_step_moves_by_lr_times_sign():
    """Bias correction makes the first Adam step lr g / (|g| + eps): lr sign(g)
    wherever |g| >> eps, whatever the scale of g (Kingma & Ba, 2015, Sec. 3)."""
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal(5000)
    g = rng.standard_normal(5000) * 10.0 ** rng.uniform(-4, 3, 5000)
    lr = 1e-3
    p1, m, v = C.adam_step(p0, np.zeros_like(p0), np.zeros_like(p0), g, 1, lr)
    assert np.allclose(p0 - p1, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    big = np.abs(g) > 1e-4
    assert big.sum() > 4000
    assert np.allclose(np.abs(p0 - p1)[big], lr, rtol=1e-3)
    assert np.array_equal(np.sign(p0 - p1), np.sign(g))


def test_adam_constant_and_alternating_gradients():
    """With a constant gradient the bias-corrected moments are exactly g and g^2,
    so every step moves by lr g / (|g| + eps).  With g then -g, the second
    corrected first moment is -(1 - b1) g / (1 + b1) while the second moment
    stays g^2: the step goes back by lr (1 - b1) / (1 + b1) sign(g).  A zero
    gradient from zero moments does not move."""
    rng = np.random.default_rng(2)
    g = rng.standard_normal(1000) * 10.0 ** rng.uniform(-3, 2, 1000)
    lr, b1 = 2e-3, 0.9
    p = np.zeros(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    for t in range(1, 8):
        pn, m, v = C.adam_step(p, m, v, g, t, lr)
        assert np.allclose(p - pn, lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)
        p = pn
    p1, m1, v1 = C.adam_step(np.zeros(1000), np.zeros(1000), np.zeros(1000), g, 1, lr)
    p2, _, _ = C.adam_step(p1, m1, v1, -g, 2, lr)
    step2 = p2 - p1
    assert np.allclose(step2, lr * (1 - b1) / (1 + b1) * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)
    z, _, _ = C.adam_step(p1, np.zeros(1000), np.zeros(1000), np.zeros(1000), 3, lr)
    assert np.array_equal(z, p1)
