"""FP64 reference of the learned warm-start network (test infrastructure:
only tests, the smoke check and the benchmark's CPU baseline use it).

The paper has no learned component; the network is a plain residual 3D CNN,
so the reference is the definition written out:

  conv(x)[v, co] = b[co] + sum_{tap, ci} xpad[v + off(tap), ci] W[tap, ci, co]

with zero padding, taps ordered tap = (dz * 3 + dy) * 3 + dx for offsets
(dz - 1, dy - 1, dx - 1), layers 4 -> 16 -> 32 -> 64 -> 2 channels (or any
widths given), ReLU after every layer but the last, and the loss
mean_v sum_c (pred - target)^2.  Gradients follow the chain rule; the tests
pin them with central finite differences.
"""
from __future__ import annotations

import itertools

import numpy as np

WIDTHS = (4, 16, 32, 64, 2)
TAPS = list(itertools.product(range(3), repeat=3))  # (dz, dy, dx), tap = (dz*3+dy)*3+dx


def unflatten(params, widths=WIDTHS):
    """Split the flat parameter vector into [(W [27, cin, cout], b [cout])]."""
    out, off = [], 0
    for cin, cout in zip(widths[:-1], widths[1:]):
        W = params[off:off + 27 * cin * cout].reshape(27, cin, cout)
        off += 27 * cin * cout
        b = params[off:off + cout]
        off += cout
        out.append((W, b))
    assert off == params.size
    return out


def n_params(widths=WIDTHS):
    return sum(27 * a * b + b for a, b in zip(widths[:-1], widths[1:]))


def conv3d(x, W, b):
    """x [Z, Y, X, cin], W [27, cin, cout], b [cout] -> [Z, Y, X, cout]."""
    Z, Y, X, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (Z, Y, X, W.shape[2])).astype(np.float64).copy()
    for tap, (dz, dy, dx) in enumerate(TAPS):
        out += xp[dz:dz + Z, dy:dy + Y, dx:dx + X, :] @ W[tap]
    return out


def conv3d_backward(x, W, g):
    """Gradients of sum(conv3d(x, W, b) * g) w.r.t. x, W and b."""
    Z, Y, X, cin = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    gflat = g.reshape(-1, g.shape[-1])
    for tap, (dz, dy, dx) in enumerate(TAPS):
        win = xp[dz:dz + Z, dy:dy + Y, dx:dx + X, :]
        gW[tap] = win.reshape(-1, cin).T @ gflat
        gxp[dz:dz + Z, dy:dy + Y, dx:dx + X, :] += g @ W[tap].T
    return gxp[1:-1, 1:-1, 1:-1, :], gW, gflat.sum(axis=0)


def forward(params, x, widths=WIDTHS, keep=False):
    """Network output [Z, Y, X, widths[-1]]; with keep, also the layer inputs."""
    layers = unflatten(params, widths)
    acts = [x]
    h = x
    for i, (W, b) in enumerate(layers):
        h = conv3d(h, W, b)
        if i + 1 < len(layers):
            h = np.maximum(h, 0.0)
        acts.append(h)
    return (h, acts) if keep else h


def loss(params, x, target, widths=WIDTHS):
    pred = forward(params, x, widths)
    V = x.shape[0] * x.shape[1] * x.shape[2]
    return float(np.sum((pred - target) ** 2) / V)


def loss_grad(params, x, target, widths=WIDTHS):
    """(loss, flat gradient) by the chain rule."""
    layers = unflatten(params, widths)
    pred, acts = forward(params, x, widths, keep=True)
    V = x.shape[0] * x.shape[1] * x.shape[2]
    L = float(np.sum((pred - target) ** 2) / V)
    g = 2.0 * (pred - target) / V
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        gx, gW, gb = conv3d_backward(acts[i], W, g)
        grads.append((gW, gb))
        if i > 0:
            g = gx * (acts[i] > 0)  # through the ReLU that produced acts[i]
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return L, np.concatenate(flat)
