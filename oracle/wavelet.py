"""Unitary periodized Daubechies-4 wavelet transform and the l1 prox (oracle,
float64; test infrastructure: only tests, the smoke check and the
benchmark's CPU baseline use it).

Sec. 2.1 lists g(x) = lambda ||Psi x||_1 with Psi a unitary wavelet transform;
Sec. 3.3.1 names the Daubechies 4 wavelet.

Readings:
  * "Daubechies 4" is the 8-tap filter with 4 vanishing moments (the naming of
    the wavelet library used by the paper's software).  The filter is derived
    here from the Daubechies spectral factorisation (minimum-phase root
    choice) rather than typed in.
  * The transform is periodized so that Psi is exactly unitary: along an axis
    of even length L, a[k] = sum_n h[n] x[(2k+n) mod L],
    d[k] = sum_n g[n] x[(2k+n) mod L] with g[n] = (-1)^n h[7-n]; the output is
    [a, d].  N-D levels apply this along every axis of the current
    approximation block (Mallat layout) and recurse on the approximation.
  * Every coefficient, the approximation included, is soft-thresholded, per
    the literal g(x) = lambda ||Psi x||_1.
  * Complex soft threshold: soft(w, tau) = w max(0, 1 - tau/|w|).
"""
from __future__ import annotations

import math

import numpy as np


def daubechies_filter(p: int = 4) -> np.ndarray:
    """Scaling filter h (length 2p) with p vanishing moments.

    |H(w)|^2 = 2 cos^{2p}(w/2) P(sin^2(w/2)), P(y) = sum_{k<p} C(p-1+k, k) y^k.
    Each root y_r of P gives a pair (zeta, 1/zeta) of roots of
    zeta^2 - (2 - 4 y_r) zeta + 1 = 0 in zeta = e^{-iw}; the minimum-phase
    filter keeps the root outside the unit circle.
    H(zeta) = const * (1 + zeta)^p * prod_r (zeta - zeta_r), normalised to
    sum h = sqrt(2).
    """
    coeffs = [math.comb(p - 1 + k, k) for k in range(p)]  # ascending in y
    yroots = np.roots(coeffs[::-1]) if p > 1 else np.array([])
    poly = np.array([1.0 + 0j])  # ascending powers of zeta
    for _ in range(p):
        poly = np.convolve(poly, [1.0, 1.0])
    for yr in yroots:
        b = 2.0 - 4.0 * yr
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zr = z1 if abs(z1) > 1.0 else z2
        poly = np.convolve(poly, [-zr, 1.0])  # (zeta - zr), ascending
    h = np.real(poly)
    h = h * (math.sqrt(2.0) / h.sum())
    return h


_H = daubechies_filter(4)


def qmf(h: np.ndarray) -> np.ndarray:
    n = np.arange(len(h))
    return ((-1.0) ** n) * h[::-1]


def _analysis_1d(x: np.ndarray, axis: int, h: np.ndarray) -> np.ndarray:
    g = qmf(h)
    x = np.moveaxis(x, axis, -1)
    L = x.shape[-1]
    half = L // 2
    a = np.zeros(x.shape[:-1] + (half,), dtype=np.complex128)
    d = np.zeros_like(a)
    for n in range(len(h)):
        idx = (2 * np.arange(half) + n) % L
        a += h[n] * x[..., idx]
        d += g[n] * x[..., idx]
    return np.moveaxis(np.concatenate([a, d], axis=-1), -1, axis)


def _synthesis_1d(c: np.ndarray, axis: int, h: np.ndarray) -> np.ndarray:
    g = qmf(h)
    c = np.moveaxis(c, axis, -1)
    L = c.shape[-1]
    half = L // 2
    a, d = c[..., :half], c[..., half:]
    x = np.zeros(c.shape, dtype=np.complex128)
    for n in range(len(h)):
        idx = (2 * np.arange(half) + n) % L
        # transpose of the analysis gather: scatter-add
        np.add.at(x, (Ellipsis, idx), h[n] * a + g[n] * d)
    return np.moveaxis(x, -1, axis)


def check_levels(shape, levels: int):
    for n in shape:
        if n % (2 ** levels) != 0:
            raise ValueError(f"axis length {n} not divisible by 2^{levels}")


def dwt(x: np.ndarray, levels: int = 4, h: np.ndarray = _H) -> np.ndarray:
    """Multi-level periodized N-D DWT in Mallat layout."""
    check_levels(x.shape, levels)
    out = np.array(x, dtype=np.complex128, copy=True)
    size = list(out.shape)
    for _ in range(levels):
        sl = tuple(slice(0, s) for s in size)
        block = out[sl]
        for ax in range(out.ndim - 1, -1, -1):  # x (last axis) first
            block = _analysis_1d(block, ax, h)
        out[sl] = block
        size = [s // 2 for s in size]
    return out


def idwt(c: np.ndarray, levels: int = 4, h: np.ndarray = _H) -> np.ndarray:
    """Inverse (= adjoint) of ``dwt``."""
    check_levels(c.shape, levels)
    out = np.array(c, dtype=np.complex128, copy=True)
    sizes = []
    size = list(out.shape)
    for _ in range(levels):
        sizes.append(list(size))
        size = [s // 2 for s in size]
    for size in reversed(sizes):
        sl = tuple(slice(0, s) for s in size)
        block = out[sl]
        for ax in range(out.ndim):  # reverse order of the analysis
            block = _synthesis_1d(block, ax, h)
        out[sl] = block
    return out


def soft(w: np.ndarray, tau: float) -> np.ndarray:
    """soft(w, tau) = w * max(0, 1 - tau / |w|)."""
    mag = np.abs(w)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(mag > 0, np.maximum(0.0, 1.0 - tau / np.where(mag > 0, mag, 1.0)), 0.0)
    return w * scale


def prox_l1_wavelet(v: np.ndarray, tau: float, levels: int = 4) -> np.ndarray:
    """argmin_x 1/2 ||x - v||^2 + tau ||Psi x||_1 = Psi^H soft(Psi v, tau)."""
    return idwt(soft(dwt(v, levels), tau), levels)


def l1_norm(x: np.ndarray, levels: int = 4) -> float:
    return float(np.sum(np.abs(dwt(x, levels))))
