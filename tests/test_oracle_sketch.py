"""Pins for PCA virtual coils and the structured sketch (Sec. 2.3.2-2.3.3)."""
import itertools
import os

import numpy as np

import synth
from oracle import cartesian as cart
from oracle import nufft
from oracle import sketch as sk

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_splitmix64_reference_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [sk.splitmix64_output(0, n) for n in (1, 2, 3)] == vals


def test_rademacher_signs_balanced_and_fresh_per_iteration():
    r = [sk.rademacher(12345, t, 6, 26) for t in range(1, 41)]
    allv = np.concatenate([a.ravel() for a in r])
    assert set(np.unique(allv)) == {-1, 1}
    assert abs(allv.mean()) < 0.05
    assert not np.array_equal(r[0], r[1])
    assert np.array_equal(r[3], sk.rademacher(12345, 4, 6, 26))


def _problem(seed=0, C=6, n=24):
    shape = (n, n)
    x = synth.phantom(shape, seed + 1)
    maps = synth.coil_maps(shape, C, seed + 2)
    mask = synth.mask_1d_vd(n, n, seed + 3, n_center=6, accel=2)
    y = cart.forward(x, maps, mask).reshape(-1, C)
    return shape, x, maps, mask, y


def test_pca_properties():
    shape, x, maps, mask, y = _problem()
    R = sk.covariance(y)
    lam, U = sk.pca(R)
    nR = np.linalg.norm(R)
    assert np.linalg.norm(R @ U - U * lam[None, :]) < 1e-12 * nR
    assert np.linalg.norm(U.conj().T @ U - np.eye(U.shape[0])) < 1e-12
    assert np.all(np.diff(lam) <= 0)
    assert abs(lam.sum() - np.sum(np.abs(y) ** 2)) < 1e-10 * lam.sum()
    kv = sk.virtual_data(y, U)
    G = kv.conj().T @ kv   # virtual channels orthogonal, energies = lambda
    assert np.linalg.norm(G - np.diag(lam)) < 1e-10 * lam.sum()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        assert abs(U[i, j].imag) < 1e-14 and U[i, j].real > 0


def test_virtual_maps_and_virtual_data_describe_one_measurement():
    # the coil rotation commutes with the per-coil operator: measuring x with
    # the virtual maps U^H c gives the virtual data U^H k of the same x, for
    # the Cartesian and the non-Cartesian operator
    shape, x, maps, mask, y = _problem(11, C=5)
    C = maps.shape[-1]
    lam, U = sk.pca(sk.covariance(y))
    vm = sk.virtual_maps(maps, U)
    a = cart.forward(x, vm, mask).reshape(-1, C)
    b = sk.virtual_data(y, U)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
    coords = synth.radial_traj(24, 6)
    plan = nufft.Plan(shape, coords, synth.radial_dcf(coords, 24))
    a = plan.forward(x, vm)
    b = sk.virtual_data(plan.forward(x, maps), U)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_covariance_undoes_the_density_weights():
    # y = w^1/2 * k: the covariance is that of the raw samples k, and samples
    # with w = 0 (which carry no information about k) are left out
    shape = (16, 16)
    maps = synth.coil_maps(shape, 4, 51)
    x = synth.phantom(shape, 52)
    coords = synth.radial_traj(16, 8)
    w = synth.radial_dcf(coords, 16).copy()
    w[::7] = 0.0
    k = nufft.Plan(shape, coords, None).forward(x, maps)
    y = nufft.Plan(shape, coords, w).forward(x, maps)
    keep = w > 0
    ref = k[keep].T @ np.conj(k[keep])
    R = sk.covariance(y, w)
    assert np.max(np.abs(R - ref)) < 1e-12 * np.max(np.abs(ref))


def test_rotation_invariance_cartesian_and_nufft():
    shape, x, maps, mask, y = _problem(5)
    lam, U = sk.pca(sk.covariance(y))
    vm = sk.virtual_maps(maps, U)
    z = _rand(shape, 1)
    a = cart.normal(z, maps, mask)
    b = cart.normal(z, vm, mask)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))
    coords = synth.radial_traj(24, 6)
    plan = nufft.Plan(shape, coords, synth.radial_dcf(coords, 24))
    a = plan.normal(z, maps)
    b = plan.normal(z, vm)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_v_equals_c_reduces_exactly():
    shape, x, maps, mask, y = _problem(7)
    C = maps.shape[-1]
    lam, U = sk.pca(sk.covariance(y))
    vm = sk.virtual_maps(maps, U)
    sm, _ = sk.sketch_for_iteration(vm, C, 0, 99, 1)
    z = _rand(shape, 2)
    a = cart.normal(z, maps, mask)
    b = cart.normal(z, sm, mask)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_exact_expectation_over_all_sign_patterns():
    # E over every Rademacher pattern of N_S equals N (E[S~^T S~] = I)
    shape, x, maps, mask, y = _problem(9, C=5, n=16)
    C, V, S = 5, 2, 2
    lam, U = sk.pca(sk.covariance(y))
    vm = sk.virtual_maps(maps, U)
    z = _rand(shape, 3)
    ref = cart.normal(z, maps, mask)
    acc = np.zeros_like(ref)
    pats = list(itertools.product([-1, 1], repeat=S * (C - V)))
    for p in pats:
        St = sk.sketch_matrix(V, S, C, np.array(p).reshape(S, C - V))
        acc += cart.normal(z, sk.sketched_maps(vm, St), mask)
    acc /= len(pats)
    assert np.max(np.abs(acc - ref)) < 1e-12 * np.max(np.abs(ref))


def test_sketch_matrix_structure():
    s = sk.rademacher(1, 1, 3, 5)
    St = sk.sketch_matrix(2, 3, 7, s)
    assert St.shape == (5, 7)
    assert np.array_equal(St[:2, :2], np.eye(2))
    assert np.all(St[:2, 2:] == 0) and np.all(St[2:, :2] == 0)
    assert np.allclose(np.abs(St[2:, 2:]), 1 / np.sqrt(3))


def test_gaussian_draw_is_standard_normal():
    from scipy import stats
    vals = np.concatenate([sk.gaussian(11, t, 32, 64).ravel() for t in range(1, 9)])
    assert vals.size == 8 * 32 * 64
    assert abs(vals.mean()) < 0.03 and abs(vals.var() - 1.0) < 0.04
    assert stats.kstest(vals, "norm").pvalue > 1e-3
    # different outer iterations and seeds draw different blocks
    assert not np.array_equal(sk.gaussian(11, 1, 2, 3), sk.gaussian(11, 2, 2, 3))
    assert not np.array_equal(sk.gaussian(11, 1, 2, 3), sk.gaussian(12, 1, 2, 3))


def test_gaussian_sketch_is_isotropic_in_expectation():
    # E[S~^T S~] = I with variance-1/S entries (averaged over many draws)
    V, S, C = 2, 3, 8
    acc = np.zeros((C, C))
    n = 3000
    for t in range(1, n + 1):
        St = sk.sketch_matrix(V, S, C, sk.gaussian(5, t, S, C - V))
        acc += St.T @ St
    assert np.max(np.abs(acc / n - np.eye(C))) < 0.1


def test_s0_diverges_where_s1_converges():
    # Sec. 3.2 reports that V = C^ (S = 0, coil compression inside the
    # subproblem) makes the sketched iteration diverge while S >= 1 designs
    # converge: l2, C^ = 4 of 8 coils
    from oracle import l2
    shape, C, lam = (32, 32), 8, 1e-2
    x = synth.phantom(shape, 21)
    maps = synth.coil_maps(shape, C, 22)
    mask = synth.mask_1d_vd(32, 32, 23, n_center=6, accel=2)
    y = cart.forward(x, maps, mask) + 1e-3 * synth.complex_noise(shape + (C,), 1.0, 24) * \
        mask[..., None]
    b = cart.adjoint(y, maps, mask)
    nfn = lambda v, m: cart.normal(v, m, mask)
    ref = l2.l2_full(lambda v: cart.normal(v, maps, mask), b, np.zeros(shape, complex), lam, 300)
    err = {}
    for V, S, dist in ((4, 0, "rademacher"), (3, 1, "rademacher"), (3, 1, "gaussian")):
        e = []
        l2.l2_sketch(nfn, maps, y.reshape(-1, C), None, b, np.zeros(shape, complex), V, S, 3, 15,
                     50, lam, dist=dist,
                     callback=lambda t, xx: e.append(np.linalg.norm(xx - ref) / np.linalg.norm(ref)))
        err[(V, S, dist)] = e
    e0 = err[(4, 0, "rademacher")]
    assert e0[-1] > 3 * min(e0)  # moves away from the minimizer
    for key in ((3, 1, "rademacher"), (3, 1, "gaussian")):
        assert err[key][-1] < 1e-3, (key, err[key])
