"""Property-based checks of the oracle over randomly drawn small problems
(hypothesis): identities that hold for every shape, trajectory and draw, so
that a mistake which only shows at some sizes (an odd length, a sample on a
grid edge, a coil count of one) fails here.

* NUFFT (Sec. 2.1, Eq. 5): the forward operator and its adjoint are adjoint
  for every trajectory, and the normal operator is their composition.
* Wavelet (the regularizer of Eq. 4): the periodized transform is unitary
  at every level count its shape admits.
* Soft threshold: it is the proximal map of tau |.| (optimality against
  perturbations), shrinks magnitudes by tau and keeps phases.
* Finite differences (l1-TV): the adjoint identity for every shape.
* Sketching matrix (Sec. 2.3.2, Eq. 13): the identity block, the +-1 /
  sqrt(S) block, and the same draw for the same (seed, iteration).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import nufft, sketch, tv, wavelet

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True)


def _crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@SETTINGS
@given(ndim=st.sampled_from([2, 3]), n=st.integers(4, 11), m_extra=st.integers(0, 3),
       nsamp=st.integers(1, 40), ncoil=st.integers(1, 3), seed=st.integers(0, 2**31 - 1))
def test_nufft_adjoint_and_normal(ndim, n, m_extra, nsamp, ncoil, seed):
    rng = np.random.default_rng(seed)
    shape = tuple([n + m_extra] + [n] * (ndim - 1)) if ndim == 3 else (n, n + m_extra)
    lim = np.array(shape[::-1], dtype=np.float64) / 2
    coords = rng.uniform(-lim, lim, size=(nsamp, ndim))
    # samples exactly on the lower edge of k-space are allowed too
    coords[0] = -lim
    dcf = rng.uniform(0.1, 2.0, nsamp)
    plan = nufft.Plan(shape, coords, dcf)
    maps = _crandn(rng, shape + (ncoil,))
    x = _crandn(rng, shape)
    y = _crandn(rng, (nsamp, ncoil))
    Ax = plan.forward(x, maps)
    AHy = plan.adjoint(y, maps)
    lhs, rhs = np.vdot(Ax, y), np.vdot(x, AHy)
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    N = plan.normal(x, maps)
    ref = plan.adjoint(Ax, maps)
    assert np.linalg.norm(N - ref) <= 1e-10 * max(1.0, np.linalg.norm(ref))
    q = np.vdot(x, N)
    assert q.real >= -1e-10 * np.linalg.norm(x) ** 2 and abs(q.imag) <= 1e-9 * max(1.0, abs(q))


@SETTINGS
@given(ndim=st.sampled_from([1, 2, 3]), levels=st.integers(1, 3),
       mults=st.lists(st.integers(1, 3), min_size=3, max_size=3), seed=st.integers(0, 2**31 - 1))
def test_wavelet_unitary(ndim, levels, mults, seed):
    rng = np.random.default_rng(seed)
    # each axis a multiple of 2^levels, at least the filter length
    shape = tuple(max(8, (2 ** levels) * k * 4) for k in mults[:ndim])
    x = _crandn(rng, shape)
    c = wavelet.dwt(x, levels)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)
    assert np.linalg.norm(wavelet.idwt(c, levels) - x) <= 1e-12 * np.linalg.norm(x)


@SETTINGS
@given(tau=st.floats(0.0, 3.0), seed=st.integers(0, 2**31 - 1), n=st.integers(1, 64))
def test_soft_threshold_is_the_prox_of_abs(tau, seed, n):
    rng = np.random.default_rng(seed)
    w = _crandn(rng, n) * rng.uniform(0.0, 3.0, n)
    z = wavelet.soft(w, tau)
    # magnitude shrinks by tau, phase kept where the result is nonzero
    assert np.allclose(np.abs(z), np.maximum(0.0, np.abs(w) - tau), atol=1e-12)
    nz = np.abs(z) > 0
    assert np.allclose(z[nz] / np.abs(z[nz]), w[nz] / np.abs(w[nz]), atol=1e-12)
    # optimality: no perturbation lowers 1/2 |z - w|^2 + tau |z| (elementwise)
    f = lambda v: 0.5 * np.abs(v - w) ** 2 + tau * np.abs(v)
    for _ in range(4):
        d = 1e-3 * _crandn(rng, n)
        assert np.all(f(z + d) >= f(z) - 1e-12)
    # non-expansive
    w2 = w + 0.1 * _crandn(rng, n)
    assert np.all(np.abs(wavelet.soft(w2, tau) - z) <= np.abs(w2 - w) + 1e-12)


@SETTINGS
@given(shape=st.lists(st.integers(1, 7), min_size=1, max_size=3), seed=st.integers(0, 2**31 - 1))
def test_finite_difference_adjoint(shape, seed):
    rng = np.random.default_rng(seed)
    x = _crandn(rng, tuple(shape))
    u = _crandn(rng, (len(shape),) + tuple(shape))
    lhs, rhs = np.vdot(tv.grad(x), u), np.vdot(x, tv.grad_adj(u))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    # constants have zero gradient (periodic differences)
    assert np.allclose(tv.grad(np.full(tuple(shape), 2.5 - 1j)), 0.0)


@SETTINGS
@given(C=st.integers(2, 12), data=st.data(), seed=st.integers(0, 2**32 - 1),
       t=st.integers(1, 1000))
def test_sketch_matrix_structure_for_every_draw(C, data, seed, t):
    V = data.draw(st.integers(0, C - 1))
    S = data.draw(st.integers(1, C - V))
    signs = sketch.rademacher(seed, t, S, C - V)
    assert set(np.unique(signs)) <= {-1, 1}
    assert np.array_equal(signs, sketch.rademacher(seed, t, S, C - V))
    St = sketch.sketch_matrix(V, S, C, signs)
    assert St.shape == (V + S, C)
    assert np.array_equal(St[:V, :V], np.eye(V)) and not St[:V, V:].any() and not St[V:, :V].any()
    assert np.allclose(np.abs(St[V:, V:]), 1.0 / np.sqrt(S))
