"""FP64 reference of the warm-start network (NumPy).

TEST INFRASTRUCTURE ONLY (oracle): the GPU kernels of the product are checked
against it; the product never imports it.  The network is not part of the
paper; it only proposes an initial state that the GLBM solve then corrects.

Tensors are channels-last (B, H, W, C).  A 3x3 convolution with periodic
padding is written as the plain sum over its nine taps:
    y[b, i, j, o] = bias[o] + sum_{dy, dx, c} w[o, c, dy+1, dx+1] x[b, i+dy, j+dx, c]
(indices modulo H and W).  Its data gradient sums the taps the other way, its
weight gradient correlates the output gradient with the shifted input.  The
network is the encoder-decoder documented in include/glbm_cnn.h.  With
bf16=True every stored activation and activation gradient is rounded to
bfloat16 (nearest even) the way the GPU stores them; arithmetic stays FP64.
"""
from __future__ import annotations

import numpy as np

# (cin, cout, relu) of the ten convolutions
SPEC = [(8, 32, True), (32, 32, True), (32, 64, True), (64, 64, True), (64, 128, True),
        (128, 128, True), (192, 64, True), (64, 64, True), (96, 32, True), (32, 3, False)]

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def round_bf16(a):
    """Nearest bfloat16 value (ties to even) of each element, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _shift(x, dy, dx):
    """s[b, i, j] = x[b, i + dy, j + dx] (periodic)."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv3x3(x, w, b=None):
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for dy, dx in TAPS:
        y += _shift(x, dy, dx) @ w[:, :, dy + 1, dx + 1].T
    if b is not None:
        y += b
    return y


def conv3x3_data_grad(gy, w):
    """dL/dx of conv3x3 given dL/dy."""
    gx = np.zeros(gy.shape[:3] + (w.shape[1],))
    for dy, dx in TAPS:
        gx += _shift(gy @ w[:, :, dy + 1, dx + 1], -dy, -dx)
    return gx


def conv3x3_weight_grad(x, gy):
    """(dL/dw, dL/db) of conv3x3 given its input x and dL/dy."""
    co, ci = gy.shape[3], x.shape[3]
    gw = np.zeros((co, ci, 3, 3))
    g2 = gy.reshape(-1, co)
    for dy, dx in TAPS:
        gw[:, :, dy + 1, dx + 1] = g2.T @ _shift(x, dy, dx).reshape(-1, ci)
    return gw, g2.sum(axis=0)


def pool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_grad(gy):
    return np.repeat(np.repeat(gy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_grad(gy):
    B, H, W, C = gy.shape
    return gy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def unpack(params):
    """Flat parameters (per layer: w [cout][cin][3][3], then b [cout]) -> list of (w, b)."""
    out, o = [], 0
    for ci, co, _ in SPEC:
        n = co * ci * 9
        w = np.asarray(params[o:o + n], dtype=np.float64).reshape(co, ci, 3, 3)
        o += n
        b = np.asarray(params[o:o + co], dtype=np.float64)
        o += co
        out.append((w, b))
    assert o == len(params)
    return out


def num_params():
    return sum(co * ci * 9 + co for ci, co, _ in SPEC)


def _perturber(perturb):
    """perturb = (rel, seed): a function that multiplies an array by 1 + rel * N(0, 1) per
    element (seeded), else the identity.  A sensitivity probe: the network evaluated
    with every convolution sum disturbed at about the FP32 rounding level shows how far
    each output moves under rounding alone."""
    if not perturb:
        return lambda a: a
    rel, seed = perturb
    rng = np.random.default_rng(seed)
    return lambda a: a * (1.0 + rel * rng.standard_normal(a.shape))


def forward(params, x, bf16=False, perturb=None):
    """Network output (B, H, W, 3) and the stored activations."""
    r = round_bf16 if bf16 else (lambda a: a)
    pt = _perturber(perturb)
    L = unpack(params)
    A = {}

    def layer(i, inp):
        w, b = L[i]
        y = pt(conv3x3(inp, w, b))
        if SPEC[i][2]:
            y = np.maximum(y, 0.0)
        return y

    A["x"] = x
    A["a0"] = r(layer(0, x))
    A["e1"] = r(layer(1, A["a0"]))
    A["p1"] = r(pool2(A["e1"]))
    A["a2"] = r(layer(2, A["p1"]))
    A["e2"] = r(layer(3, A["a2"]))
    A["p2"] = r(pool2(A["e2"]))
    A["a4"] = r(layer(4, A["p2"]))
    A["e3"] = r(layer(5, A["a4"]))
    A["c2"] = np.concatenate([A["e2"], up2(A["e3"])], axis=3)
    A["a6"] = r(layer(6, A["c2"]))
    A["d2"] = r(layer(7, A["a6"]))
    A["c1"] = np.concatenate([A["e1"], up2(A["d2"])], axis=3)
    A["a8"] = r(layer(8, A["c1"]))
    A["out"] = layer(9, A["a8"])  # FP32 output on the GPU: no bf16 rounding
    return A["out"], A


def output_abs_scale(params, A):
    """Per output element, sum_k |w_k a_k| + |bias| of the last convolution over the
    activations A of forward(): the scale against which rounding in the inputs of
    that sum is measured."""
    w, b = unpack(params)[9]
    return conv3x3(np.abs(A["a8"]), np.abs(w), np.abs(b))


def loss_and_grads(params, x, target, mask, bf16=False, abs_scale=False, perturb=None):
    """Masked MSE over channels 0..2 and its gradient with respect to the flat parameters.
    With abs_scale=True also returns, in the same flat layout, sum_pixels |dy| |x| of
    every weight and sum_pixels |dy| of every bias (the scale of each gradient's sum).
    perturb = (rel, seed) disturbs every convolution sum (forward and data gradient)
    by a relative rel (see _perturber)."""
    r = round_bf16 if bf16 else (lambda a: a)
    pt = _perturber(perturb and (perturb[0], perturb[1] + 1))
    L = unpack(params)
    out, A = forward(params, x, bf16, perturb)
    m = mask.astype(bool)
    cnt = 3.0 * m.sum()
    d = (out - target[..., :3]) * m[..., None]
    loss = float((d * d).sum() / cnt)
    gout = r(2.0 * d / cnt)
    grads = [None] * 10
    scales = [None] * 10

    def back(i, gy, inp, y):
        """Weight gradient of layer i and the gradient at its input; gy is dL/d(output)."""
        if SPEC[i][2]:
            gy = gy * (y > 0)
        grads[i] = conv3x3_weight_grad(inp, gy)
        if abs_scale:
            scales[i] = conv3x3_weight_grad(np.abs(inp), np.abs(gy))
        return pt(conv3x3_data_grad(gy, L[i][0]))

    g_a8 = r(back(9, gout, A["a8"], None))
    g_c1 = r(back(8, g_a8, A["c1"], A["a8"]))
    g_d2 = r(up2_grad(g_c1[..., 32:]))
    g_a6 = r(back(7, g_d2, A["a6"], A["d2"]))
    g_c2 = r(back(6, g_a6, A["c2"], A["a6"]))
    g_e3 = r(up2_grad(g_c2[..., 64:]))
    g_a4 = r(back(5, g_e3, A["a4"], A["e3"]))
    g_p2 = r(back(4, g_a4, A["p2"], A["a4"]))
    g_e2 = r(g_c2[..., :64] + pool2_grad(g_p2))
    g_a2 = r(back(3, g_e2, A["a2"], A["e2"]))
    g_p1 = r(back(2, g_a2, A["p1"], A["a2"]))
    g_e1 = r(g_c1[..., :32] + pool2_grad(g_p1))
    g_a0 = r(back(1, g_e1, A["a0"], A["e1"]))
    back(0, g_a0, A["x"], A["a0"])
    flat = np.concatenate([np.concatenate([gw.reshape(-1), gb]) for gw, gb in grads])
    if abs_scale:
        sflat = np.concatenate([np.concatenate([sw.reshape(-1), sb]) for sw, sb in scales])
        return loss, flat, out, sflat, A
    return loss, flat, out


def adam_step(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1) at step t >= 1, in FP64.

    m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2;
    p <- p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
    Returns the new (p, m, v); the inputs are not modified.
    """
    p, m, v, g = (np.asarray(a, dtype=np.float64) for a in (p, m, v, g))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
