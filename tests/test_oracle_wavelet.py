"""Pins for the periodized db4 transform and the l1-wavelet prox."""
import math
import os

import numpy as np

from oracle import wavelet as wv

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_filter_identities():
    h = wv.daubechies_filter(4)
    assert len(h) == 8
    assert abs(h.sum() - math.sqrt(2)) < 1e-13
    assert abs(np.sum(h * h) - 1) < 1e-13
    for k in (1, 2, 3):
        assert abs(np.sum(h[:-2 * k] * h[2 * k:])) < 1e-13
    n = np.arange(8)
    for m in range(4):
        assert abs(np.sum(((-1.0) ** n) * n ** m * h)) < 1e-10


def test_filter_closed_forms_and_table():
    # p = 1 is Haar, p = 2 has the closed form (1 +- sqrt3, 3 +- sqrt3) / (4 sqrt2)
    assert np.allclose(wv.daubechies_filter(1), [1 / math.sqrt(2)] * 2, atol=1e-15)
    s3 = math.sqrt(3)
    db2 = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * math.sqrt(2))
    assert np.max(np.abs(wv.daubechies_filter(2) - db2)) < 1e-14
    tab = np.array([float(l) for l in open(os.path.join(GOLD, "db4_daubechies1992.txt"))
                    if l.strip() and not l.startswith("#")])
    assert np.max(np.abs(wv.daubechies_filter(4) - tab)) < 1e-10


def test_unitary_2d_3d():
    for shape, L in [((32, 16), 4), ((16, 16, 32), 4), ((48, 48, 48), 4), ((20, 12), 2)]:
        x = _rand(shape, 1)
        c = wv.dwt(x, L)
        assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
        assert np.max(np.abs(wv.idwt(c, L) - x)) < 1e-12


def test_dense_matrix_orthogonal():
    shape = (16, 8)
    D = 128
    M = np.zeros((D, D))
    for j in range(D):
        e = np.zeros(D)
        e[j] = 1
        M[:, j] = wv.dwt(e.reshape(shape), 2).real.reshape(-1)
    assert np.max(np.abs(M @ M.T - np.eye(D))) < 1e-12
    # synthesis is the transpose
    c = np.random.default_rng(2).standard_normal(D)
    assert np.max(np.abs(wv.idwt(c.reshape(shape), 2).real.reshape(-1) - M.T @ c)) < 1e-12


def test_haar_level_values():
    # one level of the p=1 transform: pairwise sums / differences over sqrt2
    x = np.arange(8.0)
    c = wv._analysis_1d(x.astype(complex), 0, wv.daubechies_filter(1)).real
    a = (x[0::2] + x[1::2]) / math.sqrt(2)
    d = (x[0::2] - x[1::2]) / math.sqrt(2)
    assert np.allclose(c, np.concatenate([a, d]), atol=1e-14)


def test_soft_threshold_closed_form():
    w = np.array([3.0, -0.5, 0.0, 2 + 2j, 0.1j])
    s = wv.soft(w, 1.0)
    assert np.allclose(s, [2.0, 0.0, 0.0, (2 + 2j) * (1 - 1 / abs(2 + 2j)), 0.0])


def test_prox_optimality():
    v = _rand((32, 32), 3)
    tau = 0.7
    p = wv.prox_l1_wavelet(v, tau, 4)
    cv, cp = wv.dwt(v, 4), wv.dwt(p, 4)
    r = cv - cp
    big = np.abs(cp) > 1e-9
    # on the support, residual is tau * sign(p); elsewhere |residual| <= tau
    assert np.max(np.abs(r[big] - tau * cp[big] / np.abs(cp[big]))) < 1e-10
    assert np.max(np.abs(r[~big])) <= tau + 1e-12
