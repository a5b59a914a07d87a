"""Training and evaluation of the learned warm start (host orchestration).

Pairs come from the sketched solver itself (``Context.collect``): for outer
iteration t of Algorithm 1 the network sees (x^t / s_x, d^t / s_d) and should
predict (x^{t+1} - x^t) / s_o, where s_o = alpha rms(d^t) is the size of one
gradient step.  Training runs the library's own MFMA forward
and backward kernels on random crops of those volumes (``CNN.train_step``).
"""
from __future__ import annotations

import time

import numpy as np
import torch


def collect_pairs(problems, T, K, device="cuda"):
    """problems: iterable of (Context, y, V, S, seed, lam).  Returns lists of
    input and target volumes (one per outer iteration)."""
    ins, tgts = [], []
    for ctx, y, V, S, seed, lam in problems:
        inp, tgt, _ = ctx.collect(y, T, K, V, S, seed, lam)
        for t in range(T):
            ins.append(inp[t])
            tgts.append(tgt[t])
    return ins, tgts


def random_crop(vol_in, vol_tgt, patch, rng):
    """The same random crop of an input and a target volume (contiguous)."""
    starts = [int(rng.integers(0, max(1, s - p + 1))) for s, p in zip(vol_in.shape[:3], patch)]
    sl = tuple(slice(a, a + min(p, s)) for a, p, s in zip(starts, patch, vol_in.shape[:3]))
    return vol_in[sl].contiguous(), vol_tgt[sl].contiguous()


def train(cnn, ins, tgts, steps, patch=(32, 32, 32), lr=1e-3, seed=0, log=None):
    """Adam on random crops of random pairs; returns the per-step losses."""
    rng = np.random.default_rng(seed)
    losses = []
    for s in range(steps):
        i = int(rng.integers(0, len(ins)))
        a, b = random_crop(ins[i], tgts[i], patch, rng)
        losses.append(cnn.train_step(a, b, lr))
        if log and (s + 1) % max(1, steps // 5) == 0:
            log(f"train step {s + 1}/{steps}: loss {np.mean(losses[-20:]):.4g}")
    return losses


def evaluate(ctx, y, x_ref, cnn, T, K, V, S, seed, lam, step=0.0):
    """Plain and learned Algorithm 1 from x = 0: per-outer-iteration distance
    to x_ref and GPU time, and the warm-start decisions."""
    out = {}
    for mode in ("sketch", "learned"):
        r = ctx.recon_run(y, mode=mode, lam=lam, T=T, K=K, V=V, S=S, seed=seed, step=step,
                          x_ref=x_ref, cnn=cnn if mode == "learned" else None)
        out[mode] = {"dist": r.dist, "time_ms": r.time_ms, "alpha": r.alpha,
                     "accepted": r.n_warm_accepted, "rejected": r.n_warm_rejected,
                     "ms_warm": r.ms_warm, "x": r.x}
    return out


def time_to(dist, time_ms, thr):
    for d, t in zip(dist, time_ms):
        if d <= thr:
            return t
    return None
