"""l2 (Tikhonov) reconstruction with conjugate gradients (oracle, float64;
test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it).

Sec. 2.1 lists g(x) = lambda/2 ||x||_2^2 as a regularizer and conjugate
gradients as its solver; Sec. 3.2.2 measures the inverse g-factor of such
reconstructions by Monte Carlo.  With this g:

* ``l2_full``   -- the minimizer of 1/2 ||A x - y||^2 + lambda/2 ||x||^2
                   solves (A^H A + lambda I) x = A^H y; CG on that system.
* ``l2_sketch`` -- Algorithm 1 with this g: the subproblem of Eq. 10,
                   min_x 1/2 ||A_S (x - x^t)||^2 + <x, d> + lambda/2 ||x||^2,
                   is quadratic; with u = x - x^t it solves
                   (A_S^H A_S + lambda I) u = -(d + lambda x^t), run by CG
                   from u = 0 for K iterations.
* ``noise_std``  -- per-pixel standard deviation of a linear reconstruction
                   x = G y, G = (A^H A + lambda I)^{-1} A^H, under white
                   complex noise of unit variance on every acquired sample:
                   sqrt(diag(G G^H)) (dense, tiny problems).

Readings: CG is the textbook Hestenes-Stiefel iteration for a Hermitian
positive definite system (residual r, direction p, step <r,r>/<p,Mp>); the
inner CG starts from u = 0 at every outer iteration, as FISTA's momentum
restarts at every subproblem.
"""
from __future__ import annotations

import numpy as np

from .recon import SketchState


def cg(apply_m, rhs, x0, n_iter):
    """n_iter CG iterations on M x = rhs from x0 (M Hermitian positive
    definite, given as a function).  Stops early on an exactly zero
    residual."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = rhs - apply_m(x)
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    for _ in range(n_iter):
        if rr == 0.0:
            break
        q = apply_m(p)
        a = rr / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def l2_full(normal_fn, b, x0, lam, n_iter):
    """CG on (A^H A + lam I) x = b (b = A^H y) from x0."""
    return cg(lambda v: normal_fn(v) + lam * v, b, x0, n_iter)


def l2_sketch(normal_maps_fn, maps, y, dcf, b, x0, V, S, seed, T, K, lam, t0=1,
              callback=None, dist="rademacher"):
    """Algorithm 1 with g = lam/2 ||x||^2 and K-iteration CG inner solves.
    ``normal_maps_fn(x, maps)`` applies A^H A built on the given maps.
    Returns (x^T, state)."""
    st = SketchState(maps, y, dcf)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for t in range(t0, t0 + T):
        d = normal_maps_fn(x, maps) - b
        mt = st.maps_for(V, S, seed, t, dist)
        u = cg(lambda v: normal_maps_fn(v, mt) + lam * v, -(d + lam * x),
               np.zeros_like(x), K)
        x = x + u
        if callback is not None:
            callback(t, x)
    return x, st


def noise_std(A, lam):
    """sqrt(diag(G G^H)) with G = (A^H A + lam I)^{-1} A^H (A dense)."""
    M = A.conj().T @ A + lam * np.eye(A.shape[1])
    G = np.linalg.solve(M, A.conj().T)
    return np.sqrt(np.sum(np.abs(G) ** 2, axis=1))
