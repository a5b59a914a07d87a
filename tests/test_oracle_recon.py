"""Pins for the solvers: IHS closed form with lambda = 0, V = C reduction to
plain FISTA, the fixed point of an outer iteration, the power iteration
against the full-mask closed form, and the objective monitor's reductions
(never firing: Algorithm 1; always firing: ISTA with a monotone objective)."""
import numpy as np

import synth
from oracle import cartesian as cart
from oracle import recon
from oracle import sketch as sk
from oracle import wavelet as wv


def _rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _small(seed=0, n=16, C=6):
    shape = (n, n)
    x = synth.phantom(shape, seed + 1)
    maps = synth.coil_maps(shape, C, seed + 2)
    mask = synth.mask_1d_vd(n, n, seed + 3, n_center=4, accel=2)
    y = cart.forward(x, maps, mask) + 1e-3 * _rand(shape + (C,), seed + 4) * mask[..., None]
    return shape, x, maps, mask, y.reshape(-1, C)


def _nfn(mask):
    return lambda v, m: cart.normal(v, m, mask)


def _dense_normal(maps, mask):
    A = cart.dense_matrix(maps, mask)
    return A.conj().T @ A


def test_subproblem_lambda0_reaches_closed_form():
    # Eq. 10 with g = 0: x^{t+1} = x^t - N_S^{-1} d  (dense solve, tiny case).
    # Random (non-smooth) maps keep the sketched Hessian well conditioned.
    shape = (16, 16)
    C = 5
    maps = _rand(shape + (C,), 21)
    mask = synth.mask_1d_vd(16, 16, 4, n_center=4, accel=2)
    y = cart.forward(synth.phantom(shape, 1), maps, mask).reshape(-1, C)
    st = recon.SketchState(maps, y, None)
    ms = st.maps_for(2, 2, 7, 1)
    NS = _dense_normal(ms, mask)
    ev = np.linalg.eigvalsh(NS)
    assert ev.min() > 1e-3 * ev.max()
    xt = _rand(shape, 9)
    b = cart.adjoint(y.reshape(shape + (-1,)), maps, mask)
    d = cart.normal(xt, maps, mask) - b
    sol = xt.reshape(-1) - np.linalg.solve(NS, d.reshape(-1))
    got = recon.sketched_subproblem(lambda v: cart.normal(v, ms, mask), d, xt,
                                    1.0 / ev.max(), 0.0, 2000)
    assert np.linalg.norm(got.reshape(-1) - sol) < 1e-8 * np.linalg.norm(sol)


def test_ihs_outer_error_contracts_lambda0():
    # IHS converges geometrically in t (Sec. 2.2.2).  lambda = 0, smooth maps
    # with PCA high-energy coils; the error is measured on the well-conditioned
    # eigenspace of N (eigenvalues above 1% of the largest).
    shape = (16, 16)
    C = 6
    maps = synth.coil_maps(shape, C, 3)
    mask = synth.mask_1d_vd(16, 16, 5, n_center=4, accel=2)
    y = cart.forward(synth.phantom(shape, 2), maps, mask).reshape(-1, C)
    b = cart.adjoint(y.reshape(shape + (-1,)), maps, mask)
    w, Q = np.linalg.eigh(_dense_normal(maps, mask))
    keep = w > 1e-2 * w.max()
    Qk = Q[:, keep]
    xls = Qk @ ((Qk.conj().T @ b.reshape(-1)) / w[keep])
    errs = []

    def cb(t, xt):
        errs.append(np.linalg.norm(Qk.conj().T @ (xt.reshape(-1) - xls)))
    recon.coil_sketch(_nfn(mask), maps, y, None, b, np.zeros(shape, complex),
                      V=3, S=2, seed=3, T=7, K=200, lam=0.0, callback=cb)
    assert all(errs[i + 1] < errs[i] for i in range(6))
    assert errs[6] < 1e-2 * errs[0]


def test_v_equals_c_matches_plain_fista():
    shape, x, maps, mask, y = _small(C=5)
    C = 5
    b = cart.adjoint(y.reshape(shape + (-1,)), maps, mask)
    x0 = np.zeros(shape, complex)
    alpha, lam, K = 0.9, 1e-2, 7
    xs, _, st = recon.coil_sketch(_nfn(mask), maps, y, None, b, x0, V=C, S=0, seed=1,
                                  T=1, K=K, lam=lam, alpha=alpha)
    xf = recon.fista_full(lambda v: cart.normal(v, maps, mask), b, x0, alpha, lam, K)
    assert np.max(np.abs(xs - xf)) < 1e-12


def test_fixed_point_of_outer_iteration():
    shape, x, maps, mask, y = _small(C=6)
    b = cart.adjoint(y.reshape(shape + (-1,)), maps, mask)
    lam = 5e-3
    xinf = recon.fista_full(lambda v: cart.normal(v, maps, mask), b,
                            np.zeros(shape, complex), 1.0, lam, 3000)
    st = recon.SketchState(maps, y, None)
    for t in (1, 2):
        ms = st.maps_for(3, 2, 11, t)
        d = cart.normal(xinf, maps, mask) - b
        L = recon.power_iteration(lambda v: cart.normal(v, ms, mask), shape)
        x1 = recon.sketched_subproblem(lambda v: cart.normal(v, ms, mask), d, xinf,
                                       1.0 / L, lam, 10)
        assert np.linalg.norm(x1 - xinf) < 1e-6 * np.linalg.norm(xinf)


def test_fista_matches_its_three_sequence_form():
    # Beck and Teboulle's FISTA written the other way: x_k = prox(y_k - a g(y_k)),
    # v_k = x_{k-1} + tau_k (x_k - x_{k-1}), y_{k+1} = (1 - 1/tau_{k+1}) x_k +
    # v_k / tau_{k+1}, with tau_{k+1} the positive root of t^2 - t = tau_k^2.
    # Expanding y_{k+1} gives the momentum form the oracle uses, so the
    # iterates must agree; a wrong momentum or tau sequence breaks this.
    from oracle import wavelet as wv
    shape, x, maps, mask, y = _small(C=4)
    b = cart.adjoint(y.reshape(shape + (-1,)), maps, mask)
    N = lambda v: cart.normal(v, maps, mask)
    a, lam, K = 0.8, 5e-3, 25
    want = []
    recon.fista_full(N, b, np.zeros(shape, complex), a, lam, K, levels=2,
                     callback=lambda k, xk: want.append(xk.copy()))
    xprev = np.zeros(shape, complex)
    yk = xprev.copy()
    tau = 1.0
    for k in range(K):
        xk = wv.prox_l1_wavelet(yk - a * (N(yk) - b), a * lam, 2)
        v = xprev + tau * (xk - xprev)
        tau = max(np.roots([1.0, -1.0, -tau * tau]).real)
        yk = (1.0 - 1.0 / tau) * xk + v / tau
        xprev = xk
        assert np.max(np.abs(xk - want[k])) < 1e-12 * np.max(np.abs(want[k]))


def test_power_iteration_full_mask_closed_form():
    shape = (16, 16)
    maps = _rand(shape + (3,), 5)
    ones = np.ones(shape, np.uint8)
    L = recon.power_iteration(lambda v: cart.normal(v, maps, ones), shape, 200)
    exact = np.max(np.sum(np.abs(maps) ** 2, axis=-1))
    assert abs(L - exact) < 1e-3 * exact


def test_objective_decreases_and_nrmse():
    shape, x, maps, mask, y = _small(C=6)
    b = cart.adjoint(y.reshape(shape + (-1,)), maps, mask)
    fwd = lambda v: cart.forward(v, maps, mask).reshape(-1, 6)
    objs = []
    recon.fista_full(lambda v: cart.normal(v, maps, mask), b, np.zeros(shape, complex),
                     1.0, 1e-3, 30, callback=lambda i, xi: objs.append(recon.objective(xi, fwd, y, 1e-3)))
    assert objs[-1] < objs[0]
    assert recon.nrmse(x, x) == 0.0


def test_classical_init_with_all_coils_is_plain_fista():
    # V = C, S = 0: S^0 = U^H is unitary on the coils, so the sketched problem
    # is the full problem and the initialisation is plain FISTA
    shape, x, maps, mask, y = _small(seed=40, n=16, C=6)
    C = maps.shape[-1]
    nf = lambda v, m: cart.normal(v, m, mask)
    af = lambda yy, m: cart.adjoint(yy.reshape(shape + (m.shape[-1],)), m, mask)
    b = cart.adjoint(y.reshape(shape + (C,)), maps, mask)
    st = recon.SketchState(maps, y, None)
    alpha = 1.0 / recon.power_iteration(lambda v: nf(v, maps), shape)
    lam = 1e-3
    x1 = recon.classical_init(st, nf, af, y, np.zeros(shape, complex), C, 0, 3, 15, lam, alpha,
                              levels=2)
    ref = recon.fista_full(lambda v: nf(v, maps), b, np.zeros(shape, complex), alpha, lam, 15,
                           levels=2)
    assert np.linalg.norm(x1 - ref) < 1e-10 * np.linalg.norm(ref)


def test_classical_init_lowers_the_sketched_objective():
    # the initialisation minimises 1/2 ||S^0 A x - S^0 y||^2 + lam ||Psi x||_1
    shape, x, maps, mask, y = _small(seed=41, n=16, C=6)
    C, V, S, seed, lam = maps.shape[-1], 2, 2, 5, 1e-3
    nf = lambda v, m: cart.normal(v, m, mask)
    af = lambda yy, m: cart.adjoint(yy.reshape(shape + (m.shape[-1],)), m, mask)
    st = recon.SketchState(maps, y, None)
    m0, ent = sk.sketch_for_iteration(st.vmaps, V, S, seed, 0)
    ys = sk.virtual_data(y, st.U) @ sk.sketch_matrix(V, S, C, ent).T
    fwd = lambda v: cart.forward(v, m0, mask).reshape(-1, V + S)
    alpha = 1.0 / recon.power_iteration(lambda v: nf(v, m0), shape)
    obj = lambda v: 0.5 * np.linalg.norm(fwd(v) - ys) ** 2 + lam * recon.wv.l1_norm(v, 2)
    x1 = recon.classical_init(st, nf, af, y, np.zeros(shape, complex), V, S, seed, 40, lam,
                              alpha, levels=2)
    assert obj(x1) < 0.2 * obj(np.zeros(shape, complex))


def test_classical_init_fits_noise_free_sketched_data():
    # noise-free data y = A x_true: sketching the data gives the sketched
    # model's data of x_true (the coil mixing commutes with the operator), so
    # with lam = 0 the initialisation must drive the sketched residual
    # S^0 A (x^1 - x_true) towards zero
    shape, C, V, S, seed = (16, 16), 6, 2, 2, 5
    xt = synth.phantom(shape, 43)
    maps = synth.coil_maps(shape, C, 44)
    mask = synth.mask_1d_vd(16, 16, 45, n_center=4, accel=2)
    y = cart.forward(xt, maps, mask).reshape(-1, C)
    nf = lambda v, m: cart.normal(v, m, mask)
    af = lambda yy, m: cart.adjoint(yy.reshape(shape + (m.shape[-1],)), m, mask)
    st = recon.SketchState(maps, y, None)
    m0 = sk.sketch_for_iteration(st.vmaps, V, S, seed, 0)[0]
    alpha = 1.0 / recon.power_iteration(lambda v: nf(v, m0), shape)
    x1 = recon.classical_init(st, nf, af, y, np.zeros(shape, complex), V, S, seed, 500, 0.0,
                              alpha, levels=2)
    r = cart.forward(x1 - xt, m0, mask)
    assert np.linalg.norm(r) < 2e-3 * np.linalg.norm(cart.forward(xt, m0, mask))


def test_compression_to_all_coils_changes_nothing():
    # C0 = C: the rotation onto the virtual coils is unitary, so the
    # compressed method is Algorithm 1 itself
    shape, x, maps, mask, y = _small(seed=42, n=16, C=6)
    C = maps.shape[-1]
    nf = lambda v, m: cart.normal(v, m, mask)
    af = lambda yy, m: cart.adjoint(yy.reshape(shape + (m.shape[-1],)), m, mask)
    b = cart.adjoint(y.reshape(shape + (C,)), maps, mask)
    x0 = np.zeros(shape, complex)
    xa, alpha, _ = recon.coil_sketch(nf, maps, y, None, b, x0, 2, 2, 9, 3, 4, 1e-3, levels=2)
    xb, _, _ = recon.coil_sketch_compressed(nf, af, maps, y, None, x0, C, 2, 2, 9, 3, 4, 1e-3,
                                            alpha=alpha, levels=2)
    assert np.linalg.norm(xa - xb) < 1e-10 * np.linalg.norm(xa)


def test_compressed_algorithm1_solves_the_compressed_problem():
    # C0 < C with V = C0, S = 0: the subproblem's gradient N_c(x - x^t) + d is
    # exactly the compressed problem's N_c x - b_c, so one outer iteration is
    # plain FISTA on 1/2 ||A_c x - y_c||^2 + lam ||Psi x||_1, iterate for
    # iterate; that problem differs from the uncompressed one
    shape, x, maps, mask, y = _small(seed=43, n=16, C=6)
    C0, lam, K = 4, 1e-3, 60
    nf = lambda v, m: cart.normal(v, m, mask)
    af = lambda yy, m: cart.adjoint(yy.reshape(shape + (m.shape[-1],)), m, mask)
    st = recon.SketchState(maps, y, None)
    mc, yc = recon.compress(st, y, C0)
    alpha = 1.0 / recon.power_iteration(lambda v: nf(v, mc), shape)
    ref = recon.fista_full(lambda v: nf(v, mc), af(yc, mc), np.zeros(shape, complex), alpha, lam,
                           K, levels=2)
    xs, _, _ = recon.coil_sketch_compressed(nf, af, maps, y, None, np.zeros(shape, complex), C0,
                                            C0, 0, 4, 1, K, lam, alpha=alpha, levels=2)
    assert np.linalg.norm(xs - ref) < 1e-10 * np.linalg.norm(ref)
    full = recon.fista_full(lambda v: nf(v, maps), af(y, maps), np.zeros(shape, complex), alpha,
                            lam, K, levels=2)
    assert np.linalg.norm(full - ref) > 1e-3 * np.linalg.norm(ref)


def test_objective_of_wavelet_atoms_closed_form():
    # Eqs. 3-4: 1/2 ||A x - y||^2 + lambda ||Psi x||_1.  x is a sum of two
    # wavelet atoms, x = Psi^H (c1 e_j + c2 e_k); Psi is unitary (pinned by
    # the wavelet tests), so ||Psi x||_1 = |c1| + |c2| (complex modulus) and
    # ||x||^2 = |c1|^2 + |c2|^2.  With A = I: y = 0 leaves both terms, y = x
    # only the regularizer.
    import math
    from oracle import wavelet
    shape, lv, lam = (16, 16), 2, 0.25
    c1, c2 = 3 - 4j, -1.0
    coef = np.zeros(shape, complex)
    coef[5, 9], coef[1, 2] = c1, c2
    x = wavelet.idwt(coef, levels=lv)
    ident = lambda v: v.reshape(-1)
    l1 = abs(c1) + abs(c2)            # 6; the modulus, not |re| + |im| = 8
    sq = abs(c1) ** 2 + abs(c2) ** 2  # 26
    got0 = recon.objective(x, ident, np.zeros(x.size), lam, levels=lv)
    assert math.isclose(got0, 0.5 * sq + lam * l1, rel_tol=1e-12)
    got1 = recon.objective(x, ident, x.reshape(-1), lam, levels=lv)
    assert math.isclose(got1, lam * l1, rel_tol=1e-12)


def test_objective_data_term_against_an_explicit_sum():
    # lambda = 0: the objective is half the sum over samples of |(A x - y)_i|^2
    # for a dense complex A, written out element by element
    g = np.random.default_rng(11)
    shape = (4, 4)
    A = g.standard_normal((12, 16)) + 1j * g.standard_normal((12, 16))
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    y = g.standard_normal(12) + 1j * g.standard_normal(12)
    want = 0.0
    for i in range(12):
        s = sum(A[i, j] * x.reshape(-1)[j] for j in range(16)) - y[i]
        want += s.real ** 2 + s.imag ** 2
    want *= 0.5
    got = recon.objective(x, lambda v: A @ v.reshape(-1), y, 0.0, levels=2)
    assert abs(got - want) < 1e-12 * want


def test_nrmse_hand_computed():
    # NRMSE = ||x - ref|| / ||ref|| over all entries (Sec. 3.2.1)
    import math
    assert math.isclose(recon.nrmse(np.array([1.0, 3.0]), np.array([1.0, 1.0])), math.sqrt(2),
                        rel_tol=1e-15)
    # complex entries: ||(1j, -1)|| / ||(1, 1)|| = 1
    assert math.isclose(recon.nrmse(np.array([1 + 1j, 0]), np.array([1.0, 1.0])), 1.0,
                        rel_tol=1e-15)
    # arrays of any shape are flattened: ||(3, 0, 0, 4)|| / ||(0, 0, 0, 2)|| = 5 / 2
    assert math.isclose(recon.nrmse(np.array([[3.0, 0.0], [0.0, 6.0]]),
                                    np.array([[0.0, 0.0], [0.0, 2.0]])), 2.5, rel_tol=1e-15)


def _monitored(seed, tol, alpha_scale, T=4, K=5, lam=1e-3, V=2, S=2):
    shape, x, maps, mask, y = _small(seed=seed, C=6)
    C = maps.shape[-1]
    nf = _nfn(mask)
    fwd = lambda v, m: cart.forward(v, m, mask).reshape(-1, m.shape[-1])
    b = cart.adjoint(y.reshape(shape + (C,)), maps, mask)
    st = recon.SketchState(maps, y, None)
    Ls = recon.power_iteration(lambda v: nf(v, st.maps_for(V, S, 7, 1)), shape)
    alpha = alpha_scale / Ls
    out = recon.coil_sketch_monitored(nf, fwd, maps, y, None, b, np.zeros(shape, complex),
                                      V, S, 7, T, K, lam, tol, alpha=alpha)
    return shape, maps, mask, y, b, alpha, out


def test_monitor_that_never_fires_is_algorithm1():
    # an infinite tolerance never replaces an iterate: the monitored run is
    # Algorithm 1 itself
    shape, maps, mask, y, b, alpha, (xm, _, F0, F, fell) = _monitored(50, np.inf, 1.0)
    xr, _, _ = recon.coil_sketch(_nfn(mask), maps, y, None, b, np.zeros(shape, complex),
                                 2, 2, 7, 4, 5, 1e-3, alpha=alpha)
    assert not any(fell)
    assert np.array_equal(xm, xr)
    # the objective of x^0 = 0 is 1/2 ||y||^2
    assert abs(F0 - 0.5 * np.vdot(y, y).real) <= 1e-12 * F0


def test_monitor_with_a_diverging_inner_step_is_ista():
    # a sketched step of 30/L_S makes every subproblem's FISTA diverge, so each
    # outer iterate is replaced: the run is then proximal-gradient descent
    # (ISTA) on the full problem with step 1/L, whose objective cannot rise
    # (Beck & Teboulle 2009, Lemma 2.3)
    shape, maps, mask, y, b, alpha, (xm, _, F0, F, fell) = _monitored(51, 0.0, 30.0, T=5)
    assert all(fell)
    nf = lambda v: cart.normal(v, maps, mask)
    L = recon.power_iteration(nf, shape)
    x = np.zeros(shape, complex)
    for _ in range(5):
        x = wv.prox_l1_wavelet(x - (nf(x) - b) / L, 1e-3 / L, 4)
    assert np.allclose(xm, x, rtol=0, atol=1e-12 * np.abs(x).max())
    seq = [F0] + F
    assert all(seq[i + 1] <= seq[i] * (1 + 1e-12) for i in range(len(seq) - 1))


def test_monitor_objective_expansion_matches_definition():
    # the monitor's objective expanded through the normal operator,
    # 1/2 <x, N x> - Re <x, A^H y> + 1/2 ||y||^2, equals 1/2 ||A x - y||^2
    shape, x, maps, mask, y = _small(seed=52, C=6)
    C = maps.shape[-1]
    v = _rand(shape, 53)
    r = cart.forward(v, maps, mask).reshape(-1, C) - y
    direct = 0.5 * np.vdot(r, r).real
    b = cart.adjoint(y.reshape(shape + (C,)), maps, mask)
    expanded = (0.5 * np.vdot(v, cart.normal(v, maps, mask)).real - np.vdot(v, b).real
                + 0.5 * np.vdot(y, y).real)
    assert abs(direct - expanded) <= 1e-10 * direct
