"""Pins for the non-Cartesian oracle: brute-force NDFT of Eq. 1, KB Fourier
transform by quadrature, adjointness, dense-matrix consistency."""
import math

import numpy as np
from scipy import integrate

import synth
from oracle import nufft
from oracle import cartesian as cart


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_beta_value():
    # Beatty et al. 2005 formula for W = 4, sigma = 1.25
    b = nufft.kb_beta(4, 1.25)
    assert abs(b - math.pi * math.sqrt(10.24 * 0.5625 - 0.8)) < 1e-13
    assert 6.99 < b < 7.0


def test_kb_fourier_transform_by_quadrature():
    W, beta = 4, nufft.kb_beta(4, 1.25)
    for nu in [0.0, 0.05, 0.17, 0.31, 0.4, 0.55]:
        val, _ = integrate.quad(lambda t: nufft.kb_kernel(t, W, beta) * math.cos(2 * math.pi * nu * t),
                                -W / 2, W / 2, epsabs=1e-13, epsrel=1e-13, limit=200)
        assert abs(nufft.kb_ft(nu, W, beta) - val) < 1e-9 * abs(val)


def _ndft_err(shape, coords, W, sigma=1.25, seed=0):
    x = _rand(shape, seed)
    maps = np.ones(shape + (1,))
    plan = nufft.Plan(shape, coords, None, sigma=sigma, W=W)
    y = plan.forward(x, maps)
    ref = nufft.ndft_forward(x, maps, coords)
    return np.linalg.norm(y - ref) / np.linalg.norm(ref)


def test_against_brute_force_ndft_2d_and_3d():
    g = np.random.default_rng(1)
    c2 = g.uniform(-8, 8, size=(500, 2))
    errs = [_ndft_err((16, 16), c2, W) for W in (4, 6, 8)]
    assert errs[0] < 1e-2
    assert errs[0] > errs[1] > errs[2]
    # 3D: the per-axis KB error adds up (about 1.4e-2 at W = 4, sigma = 1.25)
    c3 = np.stack([g.uniform(-6, 6, 400), g.uniform(-5, 5, 400), g.uniform(-4, 4, 400)], 1)
    e3 = [_ndft_err((8, 10, 12), c3, W) for W in (4, 6, 8)]
    assert e3[0] < 2e-2 and e3[0] > e3[1] > e3[2]


def test_integer_k_reproduces_centred_dft():
    n = 12
    x = _rand((n, n), 3)
    ky, kx = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    coords = np.stack([kx.ravel(), ky.ravel()], 1).astype(float)
    plan = nufft.Plan((n, n), coords, None)
    y = plan.forward(x, np.ones((n, n, 1)))[:, 0].reshape(n, n)
    # centred image coordinates: DFT of the ifftshifted image, indices k mod n
    ref = np.fft.fft2(np.fft.ifftshift(x), norm="ortho")
    ref = ref[np.mod(ky, n), np.mod(kx, n)]
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-2


def test_adjointness_and_dense_normal():
    shape = (4, 4, 4)
    g = np.random.default_rng(2)
    coords = g.uniform(-2, 2, size=(60, 3))
    dcf = g.uniform(0.5, 1.5, size=60)
    maps = _rand(shape + (4,), 4)
    plan = nufft.Plan(shape, coords, dcf)
    D = 64
    A = np.zeros((60 * 4, D), dtype=complex)
    for j in range(D):
        e = np.zeros(D, complex)
        e[j] = 1
        A[:, j] = plan.forward(e.reshape(shape), maps).reshape(-1)
    y = _rand((60, 4), 5)
    AHy = plan.adjoint(y, maps).reshape(-1)
    assert np.max(np.abs(A.conj().T @ y.reshape(-1) - AHy)) < 1e-12 * np.max(np.abs(AHy))
    x = _rand(shape, 6)
    N = plan.normal(x, maps).reshape(-1)
    assert np.max(np.abs(A.conj().T @ (A @ x.reshape(-1)) - N)) < 1e-12 * np.max(np.abs(N))
    q = np.vdot(x.reshape(-1), N)
    assert abs(q.imag) < 1e-12 * abs(q) and q.real > 0


def test_interp_spread_are_transposes():
    g = np.random.default_rng(7)
    coords = g.uniform(-10, 10, size=(300, 2))
    plan = nufft.Plan((20, 24), coords, None)
    G = _rand(plan.gshape + (3,), 8)
    v = _rand((300, 3), 9)
    lhs = np.vdot(plan.interp(G), v)
    rhs = np.vdot(G, plan.spread(v))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_kb_partition_of_unity_sum():
    # interpolating a constant grid: sum of the W^d tap weights at any
    # position equals the sampled kernel sum, which is close to Phi(0)
    W, beta = 4, nufft.kb_beta(4, 1.25)
    u = np.linspace(0, 1, 17)
    s = sum(nufft.kb_kernel(u - (np.floor(u) - 1 + j), W, beta) for j in range(W))
    assert np.max(np.abs(s / nufft.kb_ft(0.0, W, beta) - 1)) < 5e-3
