"""Cartesian multi-coil SENSE operator (oracle, float64; test infrastructure:
only tests, the smoke check and the benchmark's CPU baseline use it).

Sec. 2.1, Eq. 2: k = F C x with F = I_C (x) F~ and, for Cartesian imaging,
F~ = U F~_u: the unitary DFT followed by a 0/1 undersampling.  Following the
paper's statement that U is N x N, the data is held zero-filled on the full
grid (N = D).

Reading: the DFT is the plain non-centred unitary DFT (index 0 is DC in both
image and k-space); masks are given in that layout.  The normal operator
A^H A does not depend on the choice of centring.

Layouts: image ``x`` has the image shape; maps are ``shape + (C,)``; data
``y`` is ``shape + (C,)`` (coil fastest).
"""
from __future__ import annotations

import numpy as np


def _axes(x):
    return tuple(range(x.ndim))


def forward(x: np.ndarray, maps: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """y_c = U F (c_c * x) for every coil (Eq. 2 with F~ = U F~_u)."""
    z = maps * x[..., None]
    axes = tuple(range(x.ndim))
    Z = np.fft.fftn(z, axes=axes, norm="ortho")
    return Z * mask[..., None]


def adjoint(y: np.ndarray, maps: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """x = sum_c conj(c_c) * F^H U^T y_c (adjoint of ``forward``)."""
    axes = tuple(range(maps.ndim - 1))
    z = np.fft.ifftn(y * mask[..., None], axes=axes, norm="ortho")
    return np.sum(np.conj(maps) * z, axis=-1)


def normal(x: np.ndarray, maps: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """A^H A x = sum_c conj(c_c) F^H U F (c_c x)  (U^T U = diag(mask))."""
    return adjoint(forward(x, maps, mask), maps, mask)


def dense_matrix(maps: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Explicit matrix of A (rows ordered [k][c]) for tiny problems, built from
    the DFT definition e^{-2 pi i k.r / n} / sqrt(n) per axis."""
    shape = maps.shape[:-1]
    C = maps.shape[-1]
    mats = []
    for n in shape:
        k = np.arange(n)
        mats.append(np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n))
    F = mats[0]
    for m in mats[1:]:
        F = np.kron(F, m)
    D = F.shape[0]
    mflat = mask.reshape(D).astype(float)
    cflat = maps.reshape(D, C)
    A = np.zeros((D * C, D), dtype=np.complex128)
    for c in range(C):
        A[c::C, :] = (mflat[:, None] * F) * cflat[:, c][None, :]
    return A
