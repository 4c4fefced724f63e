"""Learned source-iteration preconditioner: the network and its training step
(oracle, NumPy FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper has no learned component (it leaves the strongly scattering regime
open); the network here follows the project's own definition, written out
plainly so that the GPU kernels can be checked against it:

* Input: a structured grid of elements (nz, ny, nx) with 3 channels --
  x0 = element-average scalar-flux residual divided by its maximum modulus,
  x1 = log(sigma_t) / 5, x2 = scattering ratio c.
* U-Net of 3x3x3 convolutions (zero padding 1) with widths (c0, c1, c2):
    L0: conv(3->c0) act, conv(c0->c0) act                      -> s0
    L1: conv(c0->c1, stride 2) act, conv(c1->c1) act          -> s1
    L2: conv(c1->c2, stride 2) act, conv(c2->c2) act, conv(c2->c2) act
    up: conv(c2->c1) act at L2, nearest x2 upsample (cropped) + s1,
        conv(c1->c1) act
    up: conv(c1->c0) act at L1, nearest x2 upsample (cropped) + s0,
        conv(c0->c0) act
    out: conv(c0->1), no activation
  act = leaky ReLU with slope 0.1; every conv has a bias.
* Loss: mean squared error against the normalised target.

Convolution ("cross-correlation", as in the usual deep-learning definition):
  y[b, o, z, y, x] = bias[o] + sum_{i, kz, ky, kx} w[o, i, kz, ky, kx]
                     * x[b, i, s z + kz - 1, s y + ky - 1, s x + kx - 1]
with out-of-range input values taken as zero and output size
floor((n - 1) / s) + 1 per axis.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.1


def out_size(n: int, s: int) -> int:
    return (n - 1) // s + 1


def conv3d(x, w, b, s):
    """x (B, I, Z, Y, X), w (O, I, 3, 3, 3), b (O,) -> (B, O, Zo, Yo, Xo)."""
    B, I, Z, Y, X = x.shape
    O = w.shape[0]
    Zo, Yo, Xo = out_size(Z, s), out_size(Y, s), out_size(X, s)
    xp = np.zeros((B, I, Z + 2, Y + 2, X + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((B, O, Zo, Yo, Xo)) + b[None, :, None, None, None]
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                patch = xp[:, :, kz:kz + s * (Zo - 1) + 1:s, ky:ky + s * (Yo - 1) + 1:s,
                           kx:kx + s * (Xo - 1) + 1:s]
                y += np.einsum("oi,bizyx->bozyx", w[:, :, kz, ky, kx], patch)
    return y


def conv3d_backward(x, w, s, dy):
    """Gradients of conv3d with respect to x, w and b given dy."""
    B, I, Z, Y, X = x.shape
    _, O, Zo, Yo, Xo = dy.shape
    xp = np.zeros((B, I, Z + 2, Y + 2, X + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                sl = (slice(None), slice(None), slice(kz, kz + s * (Zo - 1) + 1, s),
                      slice(ky, ky + s * (Yo - 1) + 1, s), slice(kx, kx + s * (Xo - 1) + 1, s))
                dw[:, :, kz, ky, kx] = np.einsum("bozyx,bizyx->oi", dy, xp[sl])
                dxp[sl] += np.einsum("oi,bozyx->bizyx", w[:, :, kz, ky, kx], dy)
    db = dy.sum(axis=(0, 2, 3, 4))
    return dxp[:, :, 1:-1, 1:-1, 1:-1], dw, db


def act(v):
    return np.where(v > 0, v, SLOPE * v)


def act_backward(y, dy):
    """Leaky ReLU derivative from the activation's output (same sign as its input)."""
    return np.where(y > 0, dy, SLOPE * dy)


def upsample_add(low, skip):
    """Nearest-neighbour x2 upsample of low, cropped to skip's size, plus skip."""
    Z, Y, X = skip.shape[2:]
    up = low.repeat(2, axis=2).repeat(2, axis=3).repeat(2, axis=4)[:, :, :Z, :Y, :X]
    return up + skip


def upsample_add_backward(low_shape, dy):
    """(d low, d skip) of upsample_add."""
    B, C, z, y, x = low_shape
    Z, Y, X = dy.shape[2:]
    pad = np.zeros((B, C, 2 * z, 2 * y, 2 * x))
    pad[:, :, :Z, :Y, :X] = dy
    dlow = pad.reshape(B, C, z, 2, y, 2, x, 2).sum(axis=(3, 5, 7))
    return dlow, dy


# layer list: (name, cin, cout, stride, activation)
def layer_specs(widths):
    c0, c1, c2 = widths
    return [("e0a", 3, c0, 1, True), ("e0b", c0, c0, 1, True),
            ("e1a", c0, c1, 2, True), ("e1b", c1, c1, 1, True),
            ("e2a", c1, c2, 2, True), ("e2b", c2, c2, 1, True), ("e2c", c2, c2, 1, True),
            ("u1a", c2, c1, 1, True), ("u1b", c1, c1, 1, True),
            ("u0a", c1, c0, 1, True), ("u0b", c0, c0, 1, True),
            ("out", c0, 1, 1, False)]


def n_params(widths) -> int:
    return sum(o * i * 27 + o for _, i, o, _, _ in layer_specs(widths))


def init_params(widths, seed):
    """He-style uniform initialisation; biases zero.  Parameter vector order:
    per layer, weights (O, I, 3, 3, 3) then bias (O)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, i, o, _, a in layer_specs(widths):
        bound = np.sqrt(6.0 / (i * 27)) * (1.0 if a else 0.1)
        parts.append(rng.uniform(-bound, bound, size=o * i * 27))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def unpack(theta, widths):
    out = {}
    k = 0
    for name, i, o, s, a in layer_specs(widths):
        w = theta[k:k + o * i * 27].reshape(o, i, 3, 3, 3)
        k += o * i * 27
        b = theta[k:k + o]
        k += o
        out[name] = (w, b, s, a)
    assert k == len(theta)
    return out


def forward(theta, widths, x):
    """Returns the output (B, 1, Z, Y, X) and the cache for backward."""
    P = unpack(theta, widths)
    cache = {}

    def run(name, inp):
        w, b, s, a = P[name]
        y = conv3d(inp, w, b, s)
        if a:
            y = act(y)
        cache[name] = (inp, y)
        return y

    h = run("e0a", x)
    s0 = run("e0b", h)
    h = run("e1a", s0)
    s1 = run("e1b", h)
    h = run("e2a", s1)
    h = run("e2b", h)
    h = run("e2c", h)
    h = run("u1a", h)
    cache["up1"] = h.shape
    h = upsample_add(h, s1)
    h = run("u1b", h)
    h = run("u0a", h)
    cache["up0"] = h.shape
    h = upsample_add(h, s0)
    h = run("u0b", h)
    y = run("out", h)
    return y, cache


def backward(theta, widths, cache, dy, return_dx=False):
    """Gradient of sum(dy * forward(x)) with respect to theta (same order);
    with return_dx also the gradient with respect to the input x."""
    P = unpack(theta, widths)
    grads = {}

    def back(name, g):
        w, b, s, a = P[name]
        inp, y = cache[name]
        if a:
            g = act_backward(y, g)
        dx, dw, db = conv3d_backward(inp, w, s, g)
        grads[name] = (dw, db)
        return dx

    g = back("out", dy)
    g = back("u0b", g)
    g_low, g_s0 = upsample_add_backward(cache["up0"], g)
    g = back("u0a", g_low)
    g = back("u1b", g)
    g_low, g_s1 = upsample_add_backward(cache["up1"], g)
    g = back("u1a", g_low)
    g = back("e2c", g)
    g = back("e2b", g)
    g = back("e2a", g)
    g = back("e1b", g + g_s1)
    g = back("e1a", g)
    g = back("e0b", g + g_s0)
    dx = back("e0a", g)
    parts = []
    for name, *_ in layer_specs(widths):
        dw, db = grads[name]
        parts.append(dw.reshape(-1))
        parts.append(db)
    theta_grad = np.concatenate(parts)
    return (theta_grad, dx) if return_dx else theta_grad


def mse(y, t):
    """Loss mean((y - t)^2) and its gradient with respect to y."""
    diff = y - t
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected, step count t >= 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
