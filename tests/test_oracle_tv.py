"""Pins for the l1-TV / PDHG reference: the difference operator against its
adjoint and its Fourier eigenvalues, TV of simple images, PDHG against the
least-squares closed form (lambda = 0) and against the closed-form TV
denoising of a periodic step, and Algorithm 1 with V = C against the plain
solver."""
import numpy as np

import synth
from oracle import cartesian as cart
from oracle import tv


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_grad_adjoint_and_fourier_eigenvalues():
    for shape in ((6, 8), (4, 6, 8)):
        x = _rand(shape, 1)
        u = _rand((len(shape),) + shape, 2)
        assert np.isclose(np.vdot(tv.grad(x), u), np.vdot(x, tv.grad_adj(u)), rtol=1e-12)
        # T^H T e_k = sum_a 4 sin^2(pi k_a / n_a) e_k for a Fourier mode e_k
        k = [1, 3, 2][:len(shape)]
        grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
        e = np.exp(2j * np.pi * sum(ka * g / n for ka, g, n in zip(k, grids, shape)))
        lam = sum(4 * np.sin(np.pi * ka / n) ** 2 for ka, n in zip(k, shape))
        assert np.allclose(tv.grad_adj(tv.grad(e)), lam * e)


def test_tv_of_constant_and_step_images():
    assert tv.tv_norm(np.full((5, 7), 3 + 1j)) == 0.0
    x = np.zeros((6, 10))
    x[:, 2:5] = 2.0  # two jumps of 2 along axis 1 in each of 6 rows
    assert np.isclose(tv.tv_norm(x), 6 * 2 * 2.0)


def test_pdhg_without_regularization_is_least_squares():
    n, C = 8, 4
    shape = (n, n)
    maps = _rand(shape + (C,), 3) / np.sqrt(2 * C)
    mask = synth.mask_regular(n, n, accel=2)
    y = cart.forward(synth.phantom(shape, 4), maps, mask) + 1e-2 * _rand(shape + (C,), 5) * \
        mask[..., None]
    A = cart.dense_matrix(maps, mask)
    ref = np.linalg.solve(A.conj().T @ A, A.conj().T @ y.reshape(-1))
    b = cart.adjoint(y, maps, mask)
    # with lam = 0 the dual stays 0 and PDHG is the proximal-point iteration,
    # contracting by (1/tau) / (mu_min + 1/tau) ~ 0.988 per step here
    x = tv.pdhg_full(lambda v: cart.normal(v, maps, mask), b, np.zeros(shape, complex), 0.0,
                     2000, 10)
    assert np.linalg.norm(x.ravel() - ref) < 1e-8 * np.linalg.norm(ref)


def test_pdhg_denoises_a_periodic_step_to_its_closed_form():
    # min 1/2 ||x - x0||^2 + lam TV(x) on a periodic 1D step of height h and
    # length L (n samples): for small lam the two levels move towards each
    # other by 2 lam / L and 2 lam / (n - L) (the taut-string solution)
    n, L, h, lam = 40, 12, 1.0, 0.5
    x0 = np.zeros(n, complex)
    x0[5:5 + L] = h
    ref = x0.copy()
    ref[5:5 + L] -= 2 * lam / L
    ref[:5] += 2 * lam / (n - L)
    ref[5 + L:] += 2 * lam / (n - L)
    x = tv.pdhg_full(lambda v: v, x0, np.zeros(n, complex), lam, 3000, 2)
    assert np.max(np.abs(x - ref)) < 1e-6


def test_pdhg_on_the_bilinear_saddle_problem_reaches_the_mean():
    # G = 0 and a dual radius that no iterate reaches: min_x max_u <T x, u>.
    # Its primal solutions are the constant images, and the primal update
    # x - tau T^H u keeps the mean of x (T^H u sums to zero), so PDHG must
    # converge to the constant image at the mean of x^0.  This takes the
    # extrapolation xbar = 2 x_new - x; without it the iteration circles.
    g = np.random.default_rng(9)
    x0 = g.standard_normal((8, 8)) + 1j * g.standard_normal((8, 8))
    x = tv.pdhg(lambda v, tau, xs: v, x0, 1e6, 1000, 2)
    assert np.max(np.abs(x - x0.mean())) < 1e-9 * np.max(np.abs(x0))


def test_sketch_with_all_coils_matches_the_plain_solver():
    # V = C, S = 0: the subproblem's quadratic is the full data term, so one
    # outer iteration with a long inner solve reaches the plain minimizer
    n, C = 8, 4
    shape = (n, n)
    maps = synth.coil_maps(shape, C, 6)
    mask = synth.mask_regular(n, n, accel=2)
    y = cart.forward(synth.phantom(shape, 7), maps, mask) + 1e-2 * _rand(shape + (C,), 8) * \
        mask[..., None]
    b = cart.adjoint(y, maps, mask)
    nfn = lambda v, m: cart.normal(v, m, mask)
    lam = 2e-2
    ref = tv.pdhg_full(lambda v: nfn(v, maps), b, np.zeros(shape, complex), lam, 3000, 20)
    x, _ = tv.pdhg_sketch(nfn, maps, y.reshape(-1, C), None, b, np.zeros(shape, complex), C, 0,
                          1, 1, 3000, lam, 20)
    assert np.linalg.norm(x - ref) < 1e-6 * np.linalg.norm(ref)
