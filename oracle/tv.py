"""l1 total-variation reconstruction with PDHG (oracle, float64; test
infrastructure: only tests, the smoke check and the benchmark's CPU baseline
use it).

Sec. 2.1 lists g(x) = lambda ||T x||_1 with T the first-order finite
difference operator with periodic boundary extension, solved by the primal
dual hybrid gradient method (Chambolle and Pock 2011); the data-consistency
step of PDHG is an l2-regularized least-squares problem solved with CG
(Sec. 4.2).

* ``grad`` / ``grad_adj`` -- T x = (x[i + e_a] - x[i])_a for every axis a
  (periodic), and its adjoint T^H u = sum_a (u_a[i - e_a] - u_a[i]).
* ``pdhg`` -- for min_x G(x) + lambda ||T x||_1 with a smooth quadratic G
  whose proximal map is a linear solve:
      u <- clip(u + sigma T xbar, lambda)      (prox of the conjugate of l1)
      x_new <- prox_{tau G}(x - tau T^H u)
      xbar <- 2 x_new - x,  x <- x_new
  clip projects every complex component onto the disc of radius lambda.
* ``pdhg_full`` -- G(x) = 1/2 ||A x - y||^2: prox_{tau G}(v) solves
  (A^H A + I / tau) x = b + v / tau (b = A^H y), by CG warm-started at the
  current x.
* ``pdhg_sketch`` -- Algorithm 1 with this g: the subproblem's smooth part
  G(x) = 1/2 <x - x^t, N_S (x - x^t)> + Re<x, d> has prox
  (N_S + I / tau) x = N_S x^t - d + v / tau.

Readings: anisotropic TV (the l1 norm of all difference components, each a
complex modulus); ||T||^2 <= 4 ndim, so tau = sigma = 1 / sqrt(4 ndim) meets
tau sigma ||T||^2 <= 1; theta = 1; the dual variable restarts at 0 and x^0
is the start; a fixed number of CG iterations per PDHG step.
"""
from __future__ import annotations

import numpy as np

from .l2 import cg
from .recon import SketchState


def grad(x):
    """T x, stacked along a new first axis (one component per image axis)."""
    return np.stack([np.roll(x, -1, axis=a) - x for a in range(x.ndim)])


def grad_adj(u):
    """T^H u."""
    return sum(np.roll(u[a], 1, axis=a) - u[a] for a in range(u.shape[0]))


def tv_norm(x):
    return float(np.sum(np.abs(grad(x))))


def clip(u, lam):
    m = np.abs(u)
    return u * np.minimum(1.0, lam / np.maximum(m, 1e-300))


def steps(ndim):
    s = 1.0 / np.sqrt(4.0 * ndim)
    return s, s


def pdhg(prox_g, x0, lam, n_iter, n_dim, callback=None):
    """n_iter PDHG iterations; prox_g(v, tau, x_start) returns prox_{tau G}(v)."""
    tau, sigma = steps(n_dim)
    x = np.array(x0, dtype=np.complex128, copy=True)
    xbar = x.copy()
    u = np.zeros((n_dim,) + x.shape, dtype=np.complex128)
    for k in range(n_iter):
        u = clip(u + sigma * grad(xbar), lam)
        x_new = prox_g(x - tau * grad_adj(u), tau, x)
        xbar = 2.0 * x_new - x
        x = x_new
        if callback is not None:
            callback(k, x)
    return x


def pdhg_full(normal_fn, b, x0, lam, n_iter, n_cg, callback=None):
    """PDHG on 1/2 ||A x - y||^2 + lam ||T x||_1 (b = A^H y)."""
    def prox(v, tau, xs):
        return cg(lambda w: normal_fn(w) + w / tau, b + v / tau, xs, n_cg)
    return pdhg(prox, x0, lam, n_iter, np.ndim(x0), callback)


def pdhg_sketch(normal_maps_fn, maps, y, dcf, b, x0, V, S, seed, T, K, lam, n_cg, t0=1,
                callback=None, dist="rademacher"):
    """Algorithm 1 with g = lam ||T x||_1 and K PDHG iterations per
    subproblem.  Returns (x^T, state)."""
    st = SketchState(maps, y, dcf)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for t in range(t0, t0 + T):
        d = normal_maps_fn(x, maps) - b
        mt = st.maps_for(V, S, seed, t, dist)
        xt = x.copy()
        nxt = normal_maps_fn(xt, mt)

        def prox(v, tau, xs):
            return cg(lambda w: normal_maps_fn(w, mt) + w / tau, nxt - d + v / tau, xs, n_cg)

        x = pdhg(prox, xt, lam, K, x.ndim)
        if callback is not None:
            callback(t, x)
    return x, st
