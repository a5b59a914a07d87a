"""PCA virtual coils and the structured coil sketch (oracle, float64; test
infrastructure: only tests, the smoke check and the benchmark's CPU baseline
use it).

Sec. 2.3.2 (Eqs. 11-13): the sketch S^t = S~^t (x) I_N mixes coils only, so
A_S^t = W^1/2 F C_S^t with sketched maps c^[d] = S~^t c[d] at every pixel d.
Sec. 2.3.3: S~^t = blkdiag(I_V, S~_S^t), where the V rows keep the
high-energy virtual coils obtained by PCA coil compression (Sec. 3.1, Alg. 1)
and S~_S^t in R^{S x (C-V)} has i.i.d. random entries
(Rademacher, Sec. 3.2).

Readings:
  * PCA runs on the raw samples k_i = y_i / sqrt(w_i) (samples with w_i = 0
    are skipped); R = sum_i k_i k_i^H, R = U diag(lambda) U^H with lambda sorted
    in descending order (stable in the original index for ties).
  * Eigenvector phase: the largest-magnitude component of each column is made
    real and positive (lowest index on ties).
  * Virtual maps c'[d] = U^H c[d]; the full-coil operator is unchanged by this
    unitary rotation.
  * Rademacher entries are scaled by 1/sqrt(S) (equal to the paper's +-1 at
    S = 1) so that E[S~^T S~] = I.
  * Entry (a, b) of the draw for outer iteration t is the sign of the top bit
    of SplitMix64 output number ctr + 1 for seed ``seed``, with
    ctr = (t << 32) | (a * (C - V) + b).  SplitMix64 is Steele, Lea and Flood,
    "Fast splittable pseudorandom number generators", OOPSLA 2014: the n-th
    output is mix(seed + n * 0x9E3779B97F4A7C15) with the "mix13" finaliser.
  * Gaussian entries (the other distribution of Sec. 3.2): "sigma = 1/S" is
    read as variance 1/S, the scaling that gives E[S~^T S~] = I like the
    Rademacher draw.  Entry e = a (C - V) + b takes outputs n1 = c + 1 and
    n2 = c + 2 with c = (t << 32) | 2e, the uniforms
    u1 = ((z1 >> 11) + 1) 2^-53 in (0, 1] and u2 = (z2 >> 11) 2^-53, and the
    Box-Muller value sqrt(-2 ln u1) cos(2 pi u2) (Box and Muller, 1958).
  * S = 0 with V < C keeps only the V high-energy virtual coils (coil
    compression inside the subproblem), the design the paper reports to make
    Algorithm 1 diverge.
"""
from __future__ import annotations

import numpy as np

_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_mix(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def splitmix64_output(seed: int, n: int) -> int:
    """The n-th output (n >= 1) of SplitMix64 started from state ``seed``."""
    return splitmix64_mix((seed + n * _GAMMA) & _MASK64)


def rademacher(seed: int, t: int, S: int, CmV: int) -> np.ndarray:
    """Signs (+1/-1, int8) of the S x (C - V) block for outer iteration t."""
    out = np.empty((S, CmV), dtype=np.int8)
    for a in range(S):
        for b in range(CmV):
            ctr = ((t & 0xFFFFFFFF) << 32) | (a * CmV + b)
            z = splitmix64_output(seed, ctr + 1)
            out[a, b] = -1 if (z >> 63) else 1
    return out


def covariance(y: np.ndarray, dcf: np.ndarray | None = None) -> np.ndarray:
    """R = sum_i k_i k_i^H over samples, k_i = y_i / sqrt(w_i) (w_i > 0)."""
    k = np.asarray(y, dtype=np.complex128)
    if dcf is not None:
        keep = dcf > 0
        k = k[keep] / np.sqrt(dcf[keep])[:, None]
    # R[a, b] = sum_i k_i[a] conj(k_i[b])
    return k.T @ np.conj(k)


def fix_phase(U: np.ndarray) -> np.ndarray:
    """Make the largest-|.| entry of each column real positive (first on ties)."""
    U = U.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        u = U[i, j]
        U[:, j] *= np.conj(u) / abs(u)
    return U


def pca(R: np.ndarray):
    """Eigen-decomposition sorted by descending eigenvalue, phase fixed."""
    lam, U = np.linalg.eigh(R)
    order = sorted(range(len(lam)), key=lambda j: (-lam[j], j))
    lam = lam[order]
    U = fix_phase(U[:, order])
    return lam, U


def virtual_maps(maps: np.ndarray, U: np.ndarray) -> np.ndarray:
    """c'[d] = U^H c[d] at every pixel (coil axis last)."""
    return maps @ np.conj(U)


def virtual_data(y: np.ndarray, U: np.ndarray) -> np.ndarray:
    """k'_i = U^H k_i for every sample (coil axis last)."""
    return y @ np.conj(U)


def gaussian(seed: int, t: int, S: int, CmV: int) -> np.ndarray:
    """Unit-variance normal entries (float64) of the S x (C - V) block for
    outer iteration t (Box-Muller on two SplitMix64 uniforms per entry)."""
    out = np.empty((S, CmV), dtype=np.float64)
    for a in range(S):
        for b in range(CmV):
            c = ((t & 0xFFFFFFFF) << 32) | (2 * (a * CmV + b))
            z1 = splitmix64_output(seed, c + 1)
            z2 = splitmix64_output(seed, c + 2)
            u1 = ((z1 >> 11) + 1) * 2.0 ** -53
            u2 = (z2 >> 11) * 2.0 ** -53
            out[a, b] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return out


def sketch_matrix(V: int, S: int, C: int, entries: np.ndarray | None) -> np.ndarray:
    """S~ = blkdiag(I_V, entries / sqrt(S)), shape (V + S) x C; entries are
    the +-1 signs or the unit-variance normal values of the random block."""
    St = np.zeros((V + S, C))
    St[:V, :V] = np.eye(V)
    if S > 0:
        St[V:, V:] = np.asarray(entries, dtype=np.float64) / np.sqrt(S)
    return St


def sketched_maps(vmaps: np.ndarray, St: np.ndarray) -> np.ndarray:
    """c^[d] = S~ c'[d] at every pixel (Eq. 13)."""
    return vmaps @ St.T


def sketch_for_iteration(vmaps, V, S, seed, t, dist="rademacher"):
    C = vmaps.shape[-1]
    draw = rademacher if dist == "rademacher" else gaussian
    entries = draw(seed, t, S, C - V) if S > 0 else None
    return sketched_maps(vmaps, sketch_matrix(V, S, C, entries)), entries
