"""Pins for the Cartesian oracle (Sec. 2.1, Eq. 2 with F~ = U F~_u)."""
import numpy as np

import synth
from oracle import cartesian as cart


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_matches_brute_force_dft():
    # textbook DFT sum, written out element by element (no FFT)
    ny, nx, C = 4, 6, 3
    x = _rand((ny, nx), 1)
    maps = _rand((ny, nx, C), 2)
    mask = (np.random.default_rng(3).random((ny, nx)) > 0.4).astype(np.uint8)
    y = cart.forward(x, maps, mask)
    ref = np.zeros((ny, nx, C), dtype=complex)
    for ky in range(ny):
        for kx in range(nx):
            for c in range(C):
                s = 0
                for iy in range(ny):
                    for ix in range(nx):
                        s += maps[iy, ix, c] * x[iy, ix] * np.exp(
                            -2j * np.pi * (ky * iy / ny + kx * ix / nx))
                ref[ky, kx, c] = mask[ky, kx] * s / np.sqrt(ny * nx)
    assert np.max(np.abs(y - ref)) < 1e-12


def test_parseval_and_full_mask_identity():
    shape = (16, 12)
    x = _rand(shape, 4)
    maps = synth.coil_maps(shape, 5, 2)  # RSS = 1
    ones = np.ones(shape, np.uint8)
    y = cart.forward(x, maps, ones)
    assert abs(np.linalg.norm(y) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    # full mask: N x = (sum_j |c_j|^2) x = x
    assert np.max(np.abs(cart.normal(x, maps, ones) - x)) < 1e-12


def test_adjointness_and_psd():
    shape = (10, 14)
    x = _rand(shape, 5)
    y = _rand(shape + (4,), 6)
    maps = _rand(shape + (4,), 7)
    mask = synth.mask_1d_vd(10, 14, 3, n_center=2, accel=2)
    lhs = np.vdot(cart.forward(x, maps, mask), y)
    rhs = np.vdot(x, cart.adjoint(y, maps, mask))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    q = np.vdot(x, cart.normal(x, maps, mask))
    assert abs(q.imag) < 1e-12 * abs(q) and q.real >= 0


def test_one_dimensional_mask_needs_only_y_fft():
    # F_x^H F_x = I: with a ky-only mask the normal operator is separable
    shape = (32, 20)
    x = _rand(shape, 8)
    maps = synth.coil_maps(shape, 4, 9)
    mask = synth.mask_1d_vd(32, 20, 10, n_center=8, accel=4)
    m1 = mask[:, 0].astype(float)
    z = maps * x[..., None]
    Z = np.fft.fft(z, axis=0, norm="ortho") * m1[:, None, None]
    ref = np.sum(np.conj(maps) * np.fft.ifft(Z, axis=0, norm="ortho"), axis=-1)
    assert np.max(np.abs(cart.normal(x, maps, mask) - ref)) < 1e-12


def test_dense_matrix_consistency():
    shape = (4, 4)
    maps = _rand(shape + (2,), 11)
    mask = (np.random.default_rng(12).random(shape) > 0.5).astype(np.uint8)
    A = cart.dense_matrix(maps, mask)
    x = _rand(shape, 13)
    y = cart.forward(x, maps, mask).reshape(-1)
    assert np.max(np.abs(A @ x.reshape(-1) - y)) < 1e-12
    N = A.conj().T @ A
    assert np.max(np.abs(N @ x.reshape(-1) - cart.normal(x, maps, mask).reshape(-1))) < 1e-12
