"""Pins for the l2 (Tikhonov) reference: CG against dense solves, Algorithm 1
with l2 against the closed-form minimizer, and the noise map against its
closed form and against brute-force Monte Carlo."""
import numpy as np

import synth
from oracle import cartesian as cart
from oracle import l2


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _problem(n=8, C=4, seed=0, accel=2):
    shape = (n, n)
    x = synth.phantom(shape, seed + 1)
    maps = _rand(shape + (C,), seed + 2) / np.sqrt(2 * C)
    mask = synth.mask_regular(n, n, accel=accel)
    y = cart.forward(x, maps, mask) + 1e-2 * _rand(shape + (C,), seed + 3) * mask[..., None]
    return shape, maps, mask, y


def _closed_form(maps, mask, y, lam):
    A = cart.dense_matrix(maps, mask)
    D = A.shape[1]
    return np.linalg.solve(A.conj().T @ A + lam * np.eye(D), A.conj().T @ y.reshape(-1))


def test_cg_solves_a_small_hpd_system_in_n_steps():
    g = np.random.default_rng(0)
    n = 12
    B = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    M = B.conj().T @ B + 0.5 * np.eye(n)
    rhs = g.standard_normal(n) + 1j * g.standard_normal(n)
    x = l2.cg(lambda v: M @ v, rhs, np.zeros(n, complex), n)
    assert np.allclose(x, np.linalg.solve(M, rhs), rtol=0, atol=1e-9 * np.linalg.norm(rhs))
    # the M-norm error never grows
    xs = np.linalg.solve(M, rhs)
    errs = []
    for k in range(n + 1):
        e = l2.cg(lambda v: M @ v, rhs, np.zeros(n, complex), k) - xs
        errs.append(float(np.vdot(e, M @ e).real))
    assert all(b <= a * (1 + 1e-9) + 1e-20 for a, b in zip(errs, errs[1:]))


def test_l2_full_reaches_the_closed_form():
    shape, maps, mask, y = _problem()
    lam = 0.05
    b = cart.adjoint(y, maps, mask)
    x = l2.l2_full(lambda v: cart.normal(v, maps, mask), b, np.zeros(shape, complex), lam, 64)
    ref = _closed_form(maps, mask, y, lam)
    assert np.linalg.norm(x.ravel() - ref) < 1e-9 * np.linalg.norm(ref)


def test_sketch_with_all_coils_is_one_newton_step():
    # V = C, S = 0: the subproblem is the full problem's quadratic model,
    # which is exact for l2, so one outer iteration with an exact inner solve
    # lands on the minimizer from any start
    shape, maps, mask, y = _problem(seed=5)
    C = maps.shape[-1]
    lam = 0.02
    nfn = lambda v, m: cart.normal(v, m, mask)
    b = cart.adjoint(y, maps, mask)
    x0 = _rand(shape, 9)
    x, _ = l2.l2_sketch(nfn, maps, y.reshape(-1, C), None, b, x0, C, 0, 1, 1, 64, lam)
    ref = _closed_form(maps, mask, y, lam)
    assert np.linalg.norm(x.ravel() - ref) < 1e-9 * np.linalg.norm(ref)


def test_sketched_l2_converges_to_the_full_minimizer():
    # V < C: each subproblem is only a model, but the outer iteration keeps
    # the exact gradient, so its fixed point is the full minimizer.  Smooth
    # maps, whose energy sits in a few virtual coils (with random maps a
    # +-1 combination of two comparable virtual coils can make the model
    # too poor and the iteration diverge).
    n, C = 8, 6
    shape = (n, n)
    maps = synth.coil_maps(shape, C, 13)
    mask = synth.mask_regular(n, n, accel=2)
    y = cart.forward(synth.phantom(shape, 12), maps, mask) + \
        1e-2 * _rand(shape + (C,), 14) * mask[..., None]
    lam = 0.02
    nfn = lambda v, m: cart.normal(v, m, mask)
    b = cart.adjoint(y, maps, mask)
    ref = _closed_form(maps, mask, y, lam)
    errs = []
    # V = C - 2, S = 1: the two lowest-energy virtual coils combined into one
    l2.l2_sketch(nfn, maps, y.reshape(-1, C), None, b, np.zeros(shape, complex), C - 2, 1, 7,
                 40, 64, lam,
                 callback=lambda t, x: errs.append(np.linalg.norm(x.ravel() - ref)))
    assert errs[-1] < 1e-8 * np.linalg.norm(ref)
    assert errs[-1] < 1e-3 * errs[0]


def test_noise_std_closed_forms_and_monte_carlo():
    # full sampling, lam = 0, unit root-sum-of-squares maps: A^H A = I, so the
    # reconstruction noise is white with unit variance
    n, C = 8, 4
    maps = synth.coil_maps((n, n), C, 3)
    full = np.ones((n, n), np.uint8)
    s = l2.noise_std(cart.dense_matrix(maps, full), 0.0)
    assert np.allclose(s, 1.0, atol=1e-10)
    # regular R = 2: the closed form against brute-force simulation of the
    # linear reconstruction
    shape, maps, mask, _ = _problem(n=8, C=4, seed=2)
    lam = 0.05
    A = cart.dense_matrix(maps, mask)
    s = l2.noise_std(A, lam)
    g = np.random.default_rng(4)
    trials = 4000
    acc = np.zeros(A.shape[1])
    M = A.conj().T @ A + lam * np.eye(A.shape[1])
    rows = np.repeat(mask.reshape(-1), C).astype(bool)
    for _ in range(trials):
        noise = np.zeros(A.shape[0], complex)
        noise[rows] = (g.standard_normal(rows.sum()) + 1j * g.standard_normal(rows.sum())) / np.sqrt(2)
        acc += np.abs(np.linalg.solve(M, A.conj().T @ noise)) ** 2
    mc = np.sqrt(acc / trials)
    assert np.max(np.abs(mc / s - 1)) < 0.08
