"""Reconstruction solvers (oracle, float64; test infrastructure: only tests,
the smoke check and the benchmark's CPU baseline use it).

* ``fista_full``   -- FISTA (Beck & Teboulle) on the full problem
                      min 1/2 ||A x - y||^2 + lambda ||Psi x||_1 (Eqs. 3-4,
                      regularizer 2, solver 2 of Sec. 2.1.1).
* ``coil_sketch``  -- Algorithm 1 (Sec. 2.3.4): for t = 1..T compute the true
                      gradient d = A^H (A x^t - y), form the sketched model
                      A_S^t = S^t A with C^ coils, and solve the sketched
                      subproblem (Eqs. 9-10)
                        min_x 1/2 ||A_S^t (x - x^t)||^2 + <x, d> + g(x)
                      with FISTA, whose smooth-part gradient is
                      A_S^H A_S (x - x^t) + d.
* ``power_iteration`` -- step size 1/L from the first subproblem, reused for
                      all subproblems (Sec. 3.3.1).

Readings:
  * <x, d> is Re(x^H d), whose gradient is d.
  * FISTA momentum restarts (tau = 1, z = x^t) at every subproblem.
  * The power iteration starts from the normalised all-ones image, runs 30
    normalised applies and reports L = ||N v_30||.
  * Alg. 1's initial compression keeps all C coils unless C0 < C is asked
    for (``coil_sketch_compressed``): then the model and the data are rotated
    onto the PCA virtual coils and truncated to the first C0; x^0 = 0.  The optional
    classical-sketch initialisation (off by default) uses the structured
    sketch drawn at t = 0 on both the model and the data and the same FISTA
    (step from the first subproblem) for a given number of iterations.
  * K inner FISTA iterations per subproblem.
  * ``coil_sketch_monitored`` adds an objective monitor that the paper does
    not have: F(x) = 1/2 ||A x - y||^2 + lambda ||Psi x||_1 (Eqs. 3-4) of
    x^{t0} and of each outer iterate; an iterate whose F is not finite or
    exceeds F(x^t) + tol |F(x^t)| is replaced by one proximal-gradient step
    on the full problem from x^t with step 1/L, L from the power iteration
    on the full normal operator, and the run continues from it.
"""
from __future__ import annotations

import math

import numpy as np

from . import sketch as sk
from . import wavelet as wv


def nrmse(x, ref) -> float:
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def power_iteration(normal_fn, shape, n_iter: int = 30) -> float:
    v = np.ones(shape, dtype=np.complex128)
    v /= np.linalg.norm(v.ravel())
    for _ in range(n_iter):
        w = normal_fn(v)
        v = w / np.linalg.norm(w.ravel())
    return float(np.linalg.norm(normal_fn(v).ravel()))


def objective(x, forward_fn, y, lam, levels=4) -> float:
    r = forward_fn(x) - y
    return 0.5 * float(np.vdot(r, r).real) + lam * wv.l1_norm(x, levels)


def _fista_momentum(tau):
    tau_n = (1.0 + math.sqrt(1.0 + 4.0 * tau * tau)) / 2.0
    return tau_n, (tau - 1.0) / tau_n


def fista_full(normal_fn, b, x0, alpha, lam, n_iter, levels=4, callback=None):
    """Plain FISTA on 1/2||Ax-y||^2 + lam||Psi x||_1 with gradient N x - b."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    z = x.copy()
    tau = 1.0
    for it in range(n_iter):
        g = normal_fn(z) - b
        x_new = wv.prox_l1_wavelet(z - alpha * g, alpha * lam, levels)
        tau, beta = _fista_momentum(tau)
        z = x_new + beta * (x_new - x)
        x = x_new
        if callback is not None:
            callback(it, x)
    return x


def sketched_subproblem(normal_s, d, xt, alpha, lam, K, levels=4, z0=None):
    """K FISTA steps on Eq. 10 + g: gradient N_S (z - x^t) + d."""
    x = xt.copy()
    z = xt.copy() if z0 is None else np.array(z0, dtype=np.complex128, copy=True)
    tau = 1.0
    for _ in range(K):
        g = normal_s(z - xt) + d
        x_new = wv.prox_l1_wavelet(z - alpha * g, alpha * lam, levels)
        tau, beta = _fista_momentum(tau)
        z = x_new + beta * (x_new - x)
        x = x_new
    return x


class SketchState:
    """PCA basis and virtual maps computed once per reconstruction."""

    def __init__(self, maps, y, dcf):
        self.R = sk.covariance(y, dcf)
        self.lam, self.U = sk.pca(self.R)
        self.vmaps = sk.virtual_maps(maps, self.U)

    def maps_for(self, V, S, seed, t, dist="rademacher"):
        return sk.sketch_for_iteration(self.vmaps, V, S, seed, t, dist)[0]


def classical_init(st, normal_maps_fn, adjoint_maps_fn, y, x0, V, S, seed, K0, lam, alpha,
                   levels=4, dist="rademacher"):
    """Alg. 1's optional initialisation: x^1 = argmin 1/2 ||S^0 A x - S^0 y||^2
    + g(x), with S^0 the structured sketch drawn at t = 0 applied to the
    model (sketched maps) and to the data (y -> S~^0 U^H y per sample), by
    K0 FISTA iterations from x0.  ``adjoint_maps_fn(y, maps)`` applies A^H."""
    C = st.vmaps.shape[-1]
    m0, entries = sk.sketch_for_iteration(st.vmaps, V, S, seed, 0, dist)
    St = sk.sketch_matrix(V, S, C, entries)
    ys = sk.virtual_data(y, st.U) @ St.T
    bs = adjoint_maps_fn(ys, m0)
    return fista_full(lambda v: normal_maps_fn(v, m0), bs, x0, alpha, lam, K0, levels)


def compress(st, y, C0):
    """Alg. 1's initial coil compression: the first C0 virtual maps and the
    data rotated onto them, (U^H y)[:, :C0] per sample."""
    return st.vmaps[..., :C0], sk.virtual_data(y, st.U)[:, :C0]


def coil_sketch_compressed(normal_maps_fn, adjoint_maps_fn, maps, y, dcf, x0, C0, V, S, seed,
                           T, K, lam, alpha=None, levels=4, n_pow=30, callback=None, t0=1,
                           dist="rademacher"):
    """Algorithm 1 after its initial compression to the first C0 virtual
    coils: the true gradient and the sketches both use the compressed
    model A_c (maps U^H c truncated to C0) and data y_c; V + S <= C0.
    Returns (x^T, alpha, state)."""
    st = SketchState(maps, y, dcf)
    mc, yc = compress(st, y, C0)
    bc = adjoint_maps_fn(yc, mc)
    if alpha is None:
        m1 = sk.sketch_for_iteration(mc, V, S, seed, 1, dist)[0]
        alpha = 1.0 / power_iteration(lambda v: normal_maps_fn(v, m1), x0.shape, n_pow)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for t in range(t0, t0 + T):
        d = normal_maps_fn(x, mc) - bc
        mt = sk.sketch_for_iteration(mc, V, S, seed, t, dist)[0]
        x = sketched_subproblem(lambda v: normal_maps_fn(v, mt), d, x, alpha, lam, K, levels)
        if callback is not None:
            callback(t, x)
    return x, alpha, st


def coil_sketch(normal_maps_fn, maps, y, dcf, b, x0, V, S, seed, T, K, lam,
                alpha=None, levels=4, n_pow=30, callback=None, t0=1, dist="rademacher",
                init_iters=0, adjoint_maps_fn=None):
    """Algorithm 1 with FISTA inner solves.

    ``normal_maps_fn(x, maps)`` applies A^H A built on the given maps.
    ``b`` = A^H y.  With init_iters > 0, x^1 comes from the classical-sketch
    initialisation (``adjoint_maps_fn`` needed).  Returns (x^T, alpha, state).
    """
    st = SketchState(maps, y, dcf)
    if alpha is None:
        m1 = st.maps_for(V, S, seed, 1, dist)
        L = power_iteration(lambda v: normal_maps_fn(v, m1), x0.shape, n_pow)
        alpha = 1.0 / L
    x = np.array(x0, dtype=np.complex128, copy=True)
    if init_iters > 0:
        x = classical_init(st, normal_maps_fn, adjoint_maps_fn, y, x, V, S, seed, init_iters,
                           lam, alpha, levels, dist)
    for t in range(t0, t0 + T):
        d = normal_maps_fn(x, maps) - b
        mt = st.maps_for(V, S, seed, t, dist)
        x = sketched_subproblem(lambda v: normal_maps_fn(v, mt), d, x, alpha, lam, K, levels)
        if callback is not None:
            callback(t, x)
    return x, alpha, st


def fallback_step(x, d, L, lam, levels=4):
    """The monitor's replacement iterate: one proximal-gradient step on the
    full problem from x with gradient d, prox_{lam/L}(x - d/L)."""
    return wv.prox_l1_wavelet(x - d / L, lam / L, levels)


def coil_sketch_monitored(normal_maps_fn, forward_maps_fn, maps, y, dcf, b, x0, V, S, seed,
                          T, K, lam, tol, alpha=None, levels=4, n_pow=30, t0=1,
                          dist="rademacher"):
    """Algorithm 1 (all coils, FISTA inner solves) with the objective monitor.

    ``forward_maps_fn(x, maps)`` applies A (samples x coils, the layout of
    ``y``).  Returns (x, alpha, F0, F, fell_back): F0 = F(x^{t0}), F[i] and
    fell_back[i] those of the iterate kept after outer iteration i.
    """
    st = SketchState(maps, y, dcf)
    if alpha is None:
        m1 = st.maps_for(V, S, seed, t0, dist)
        alpha = 1.0 / power_iteration(lambda v: normal_maps_fn(v, m1), x0.shape, n_pow)
    full = lambda v: normal_maps_fn(v, maps)
    F = lambda v: objective(v, lambda u: forward_maps_fn(u, maps), y, lam, levels)
    x = np.array(x0, dtype=np.complex128, copy=True)
    f_prev = F(x)
    F0 = f_prev
    L_full = None
    objs, fell = [], []
    for t in range(t0, t0 + T):
        d = full(x) - b
        mt = st.maps_for(V, S, seed, t, dist)
        x_new = sketched_subproblem(lambda v: normal_maps_fn(v, mt), d, x, alpha, lam, K, levels)
        with np.errstate(over="ignore", invalid="ignore"):
            f = F(x_new)
        bad = not np.isfinite(f) or f > f_prev + tol * abs(f_prev)
        if bad:
            if L_full is None:
                L_full = power_iteration(full, x0.shape, n_pow)
            x_new = fallback_step(x, d, L_full, lam, levels)
            f = F(x_new)
        objs.append(f)
        fell.append(bad)
        x, f_prev = x_new, f
    return x, alpha, F0, objs, fell
