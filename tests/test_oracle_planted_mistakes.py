"""The oracle's pins catch plausible mistakes.  Each case plants one error in
an oracle function (a dropped term, a wrong sign, index or scale, a
transposed or conjugated operand), on the CPU and only for the duration of
the case, and checks that a pin written against the paper or the mathematics
then fails.  A pin that still passed would not be pinning that part."""
import math

import numpy as np
import pytest

from oracle import cartesian, cnn, l2, nufft, recon, sketch, tv, wavelet
from tests import (test_oracle_cartesian as p_cart, test_oracle_cnn as p_cnn,
                   test_oracle_l2 as p_l2,
                   test_oracle_nufft as p_nufft, test_oracle_recon as p_recon,
                   test_oracle_sketch as p_sketch, test_oracle_tv as p_tv,
                   test_oracle_wavelet as p_wav)


# -- planted mistakes ---------------------------------------------------------

def cart_forward_without_mask(x, maps, mask):
    return np.fft.fftn(maps * x[..., None], axes=tuple(range(x.ndim)), norm="ortho")


def cart_forward_unnormalised(x, maps, mask):
    return np.fft.fftn(maps * x[..., None], axes=tuple(range(x.ndim))) * mask[..., None]


def cart_adjoint_without_conj(y, maps, mask):
    z = np.fft.ifftn(y * mask[..., None], axes=tuple(range(maps.ndim - 1)), norm="ortho")
    return np.sum(maps * z, axis=-1)


def cart_adjoint_wrong_exponent(y, maps, mask):
    z = np.fft.fftn(y * mask[..., None], axes=tuple(range(maps.ndim - 1)), norm="ortho")
    return np.sum(np.conj(maps) * z, axis=-1)


def kb_beta_without_offset(W, sigma):
    return math.pi * math.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2)


def deapod_at_image_frequency(shape, gshape, W, beta):
    # Phi evaluated at r / n instead of r / m (the grid's frequency)
    return _orig_deapod(shape, shape, W, beta)


_orig_deapod = nufft.deapod


def tap_iter_swapped_strides(self):
    W = self.W
    for combo in np.ndindex(*([W] * self.ndim)):
        w = np.ones(self.N)
        lin = np.zeros(self.N, dtype=np.int64)
        for a in reversed(range(self.ndim)):
            w = w * self.wts[a][:, combo[a]]
            lin = lin * self.gshape[a] + self.taps[a][:, combo[a]]
        yield lin, w


def spread_real_part_only(self, vals):
    C = vals.shape[-1]
    M = int(np.prod(self.gshape))
    out = np.zeros((M, C), dtype=np.complex128)
    for lin, w in self._tap_iter():
        for c in range(C):
            out[:, c] += np.bincount(lin, weights=w * vals[:, c].real, minlength=M)
    return out.reshape(self.gshape + (C,))


def normal_with_sqrt_weights(self, x, maps):
    z = maps * (x / self.apod)[..., None]
    v = self.interp(self.fft_grid(z)) / math.sqrt(self.D)
    v = v * self._w("sqrt")[:, None]
    out = self.ifft_grid(self.spread(v)) / math.sqrt(self.D) / self.apod[..., None]
    return np.sum(np.conj(maps) * out, axis=-1)


def sketch_matrix_unscaled(V, S, C, entries):
    St = np.zeros((V + S, C))
    St[:V, :V] = np.eye(V)
    if S > 0:
        St[V:, V:] = np.asarray(entries, dtype=np.float64)
    return St


def covariance_conjugated(y, dcf=None):
    k = np.asarray(y, dtype=np.complex128)
    return np.conj(k).T @ k


def virtual_maps_without_conj(maps, U):
    return maps @ U


def fix_phase_negative(U):
    U = _orig_fix_phase(U)
    return -U


_orig_fix_phase = sketch.fix_phase


def fista_momentum_off_by_one(tau):
    tau_n = (1.0 + math.sqrt(1.0 + 4.0 * tau * tau)) / 2.0
    return tau_n, tau / tau_n


def subproblem_wrong_sign_of_d(normal_s, d, xt, alpha, lam, K, levels=4, z0=None):
    return _orig_subproblem(normal_s, -d, xt, alpha, lam, K, levels, z0)


_orig_subproblem = recon.sketched_subproblem


def power_iteration_norm_of_v(normal_fn, shape, n_iter=30):
    v = np.ones(shape, dtype=np.complex128)
    v /= np.linalg.norm(v.ravel())
    for _ in range(n_iter):
        w = normal_fn(v)
        v = w / np.linalg.norm(w.ravel())
    return float(np.linalg.norm(v.ravel()))


def cg_inverted_beta(apply_m, rhs, x0, n_iter):
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = rhs - apply_m(x)
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    for _ in range(n_iter):
        if rr == 0.0:
            break
        q = apply_m(p)
        a = rr / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr / rr_new) * p
        rr = rr_new
    return x


def l2_full_without_lambda(normal_fn, b, x0, lam, n_iter):
    return l2.cg(normal_fn, b, x0, n_iter)


def tv_grad_backward_difference(x):
    return np.stack([np.roll(x, 1, axis=a) - x for a in range(x.ndim)])


def tv_clip_half_radius(u, lam):
    return _orig_clip(u, lam / 2)


_orig_clip = tv.clip


def qmf_without_alternation(h):
    return h[::-1].copy()


def soft_without_floor(w, tau):
    mag = np.abs(w)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(mag > 0, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
    return w * scale


def pdhg_without_extrapolation(prox_g, x0, lam, n_iter, n_dim, callback=None):
    tau, sigma = tv.steps(n_dim)
    x = np.array(x0, dtype=np.complex128, copy=True)
    u = np.zeros((n_dim,) + x.shape, dtype=np.complex128)
    for _ in range(n_iter):
        u = tv.clip(u + sigma * tv.grad(x), lam)
        x = prox_g(x - tau * tv.grad_adj(u), tau, x)
    return x


def classical_init_data_unsketched(st, normal_maps_fn, adjoint_maps_fn, y, x0, V, S, seed, K0,
                                   lam, alpha, levels=4, dist="rademacher"):
    # the model is sketched but the data only rotated and truncated
    m0, _ = sketch.sketch_for_iteration(st.vmaps, V, S, seed, 0, dist)
    ys = sketch.virtual_data(y, st.U)[:, :V + S]
    return recon.fista_full(lambda v: normal_maps_fn(v, m0), adjoint_maps_fn(ys, m0), x0,
                            alpha, lam, K0, levels)


def compress_data_unrotated(st, y, C0):
    return st.vmaps[..., :C0], np.asarray(y)[:, :C0]


def l2_sketch_without_lam_x(normal_maps_fn, maps, y, dcf, b, x0, V, S, seed, T, K, lam, t0=1,
                            callback=None, dist="rademacher"):
    # the subproblem's right-hand side loses the -lam x^t term
    st = recon.SketchState(maps, y, dcf)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for t in range(t0, t0 + T):
        d = normal_maps_fn(x, maps) - b
        mt = st.maps_for(V, S, seed, t, dist)
        x = x + l2.cg(lambda v: normal_maps_fn(v, mt) + lam * v, -d, np.zeros_like(x), K)
    return x, st


def pdhg_sketch_with_plus_d(normal_maps_fn, maps, y, dcf, b, x0, V, S, seed, T, K, lam, n_cg,
                            t0=1, callback=None, dist="rademacher"):
    # the subproblem's linear term enters with the wrong sign
    st = recon.SketchState(maps, y, dcf)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for t in range(t0, t0 + T):
        d = normal_maps_fn(x, maps) - b
        mt = st.maps_for(V, S, seed, t, dist)
        xt = x.copy()
        nxt = normal_maps_fn(xt, mt)

        def prox(v, tau, xs):
            return l2.cg(lambda w: normal_maps_fn(w, mt) + w / tau, nxt + d + v / tau, xs, n_cg)
        x = tv.pdhg(prox, xt, lam, K, x.ndim)
    return x, st


def covariance_of_weighted_samples(y, dcf=None):
    # the density weights are not divided out
    k = np.asarray(y, dtype=np.complex128)
    return k.T @ np.conj(k)


def pad_uncentred(self, z):
    # image index i placed at grid index i instead of (i - n/2) mod m
    C = z.shape[-1]
    g = np.zeros(self.gshape + (C,), dtype=np.complex128)
    g[tuple(slice(0, n) for n in self.shape)] = z
    return g


def kb_ft_with_sin_for_sinh(nu, W, beta):
    nu = np.asarray(nu, dtype=np.float64)
    a = beta ** 2 - (math.pi * W * nu) ** 2
    s = np.sqrt(np.abs(a))
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(a != 0, W * np.sin(s) / s, W)


def conv3d_mirrored_taps(x, W, b):
    # tap (dz, dy, dx) reads the mirrored offset: a correlation turned into a
    # convolution
    Z, Y, X, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (Z, Y, X, W.shape[2])).astype(np.float64).copy()
    for tap, (dz, dy, dx) in enumerate(cnn.TAPS):
        out += xp[2 - dz:2 - dz + Z, 2 - dy:2 - dy + Y, 2 - dx:2 - dx + X, :] @ W[tap]
    return out


def objective_without_half(x, forward_fn, y, lam, levels=4):
    r = forward_fn(x) - y
    return float(np.vdot(r, r).real) + lam * wavelet.l1_norm(x, levels)


def objective_with_l2_regularizer(x, forward_fn, y, lam, levels=4):
    r = forward_fn(x) - y
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.linalg.norm(wavelet.dwt(x, levels)))


def objective_with_re_im_l1(x, forward_fn, y, lam, levels=4):
    r = forward_fn(x) - y
    c = wavelet.dwt(x, levels)
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.sum(np.abs(c.real) + np.abs(c.imag)))


def nrmse_squared(x, ref):
    return float(np.linalg.norm((x - ref).ravel()) ** 2 / np.linalg.norm(ref.ravel()) ** 2)


def nrmse_over_x(x, ref):
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(x.ravel()))


def fallback_step_ascending(x, d, L, lam, levels=4):
    return wavelet.prox_l1_wavelet(x + d / L, lam / L, levels)


def fallback_step_half_threshold(x, d, L, lam, levels=4):
    return wavelet.prox_l1_wavelet(x - d / L, 0.5 * lam / L, levels)


CASES = [
    # (name, owner, attribute, planted function, pins expected to fail)
    ("cartesian forward drops the mask", cartesian, "forward", cart_forward_without_mask,
     [p_cart.test_matches_brute_force_dft]),
    ("cartesian forward drops 1/sqrt(D)", cartesian, "forward", cart_forward_unnormalised,
     [p_cart.test_matches_brute_force_dft, p_cart.test_parseval_and_full_mask_identity]),
    ("cartesian adjoint drops conj(c)", cartesian, "adjoint", cart_adjoint_without_conj,
     [p_cart.test_adjointness_and_psd]),
    ("cartesian adjoint with the forward exponent", cartesian, "adjoint",
     cart_adjoint_wrong_exponent, [p_cart.test_adjointness_and_psd]),
    ("KB beta without the -0.8", nufft, "kb_beta", kb_beta_without_offset,
     [p_nufft.test_beta_value]),
    ("deapodisation at r/n", nufft, "deapod", deapod_at_image_frequency,
     [p_nufft.test_against_brute_force_ndft_2d_and_3d]),
    ("gridding with swapped axis strides", nufft.Plan, "_tap_iter", tap_iter_swapped_strides,
     [p_nufft.test_against_brute_force_ndft_2d_and_3d]),
    ("spreading drops the imaginary part", nufft.Plan, "spread", spread_real_part_only,
     [p_nufft.test_interp_spread_are_transposes]),
    ("normal operator weighted by sqrt(w)", nufft.Plan, "normal", normal_with_sqrt_weights,
     [p_nufft.test_adjointness_and_dense_normal]),
    ("sketch without 1/sqrt(S)", sketch, "sketch_matrix", sketch_matrix_unscaled,
     [p_sketch.test_exact_expectation_over_all_sign_patterns]),
    ("covariance conjugated", sketch, "covariance", covariance_conjugated,
     [p_sketch.test_pca_properties]),
    ("virtual maps with U instead of U^H", sketch, "virtual_maps", virtual_maps_without_conj,
     [p_sketch.test_virtual_maps_and_virtual_data_describe_one_measurement]),
    ("eigenvector phase made negative", sketch, "fix_phase", fix_phase_negative,
     [p_sketch.test_pca_properties]),
    ("FISTA momentum tau/tau+ instead of (tau-1)/tau+", recon, "_fista_momentum",
     fista_momentum_off_by_one, [p_recon.test_fista_matches_its_three_sequence_form]),
    ("subproblem gradient with -d", recon, "sketched_subproblem", subproblem_wrong_sign_of_d,
     [p_recon.test_fixed_point_of_outer_iteration]),
    ("power iteration returns |v|", recon, "power_iteration", power_iteration_norm_of_v,
     [p_recon.test_power_iteration_full_mask_closed_form]),
    ("CG with the inverted beta", l2, "cg", cg_inverted_beta,
     [p_l2.test_cg_solves_a_small_hpd_system_in_n_steps]),
    ("l2 solve without lambda", l2, "l2_full", l2_full_without_lambda,
     [p_l2.test_l2_full_reaches_the_closed_form]),
    ("TV with backward differences", tv, "grad", tv_grad_backward_difference,
     [p_tv.test_grad_adjoint_and_fourier_eigenvalues]),
    ("TV dual clipped at lambda/2", tv, "clip", tv_clip_half_radius,
     [p_tv.test_pdhg_denoises_a_periodic_step_to_its_closed_form]),
    ("wavelet high-pass without (-1)^n", wavelet, "qmf", qmf_without_alternation,
     [p_wav.test_unitary_2d_3d, p_wav.test_dense_matrix_orthogonal]),
    ("soft threshold without max(0, .)", wavelet, "soft", soft_without_floor,
     [p_wav.test_soft_threshold_closed_form]),
    ("PDHG without the extrapolation", tv, "pdhg", pdhg_without_extrapolation,
     [p_tv.test_pdhg_on_the_bilinear_saddle_problem_reaches_the_mean]),
    ("classical initialisation with unsketched data", recon, "classical_init",
     classical_init_data_unsketched, [p_recon.test_classical_init_fits_noise_free_sketched_data]),
    ("compression rotates the maps but not the data", recon, "compress",
     compress_data_unrotated, [p_recon.test_compression_to_all_coils_changes_nothing]),
    ("l2 subproblem without -lam x^t", l2, "l2_sketch", l2_sketch_without_lam_x,
     [p_l2.test_sketch_with_all_coils_is_one_newton_step]),
    ("TV subproblem with +d", tv, "pdhg_sketch", pdhg_sketch_with_plus_d,
     [p_tv.test_sketch_with_all_coils_matches_the_plain_solver]),
    ("covariance of the weighted samples", sketch, "covariance",
     covariance_of_weighted_samples, [p_sketch.test_covariance_undoes_the_density_weights]),
    ("zero padding without centring", nufft.Plan, "_pad", pad_uncentred,
     [p_nufft.test_against_brute_force_ndft_2d_and_3d]),
    ("KB transform with sin for sinh", nufft, "kb_ft", kb_ft_with_sin_for_sinh,
     [p_nufft.test_kb_fourier_transform_by_quadrature]),
    ("convolution with mirrored taps", cnn, "conv3d", conv3d_mirrored_taps,
     [p_cnn.test_delta_kernel_is_identity_and_shift, p_cnn.test_conv_matches_brute_force_sum]),
    ("objective without the 1/2", recon, "objective", objective_without_half,
     [p_recon.test_objective_of_wavelet_atoms_closed_form,
      p_recon.test_objective_data_term_against_an_explicit_sum]),
    ("objective with the l2 norm of the coefficients", recon, "objective",
     objective_with_l2_regularizer, [p_recon.test_objective_of_wavelet_atoms_closed_form]),
    ("objective with |re| + |im| for the modulus", recon, "objective", objective_with_re_im_l1,
     [p_recon.test_objective_of_wavelet_atoms_closed_form]),
    ("NRMSE of squared norms", recon, "nrmse", nrmse_squared, [p_recon.test_nrmse_hand_computed]),
    ("NRMSE normalised by x", recon, "nrmse", nrmse_over_x, [p_recon.test_nrmse_hand_computed]),
    ("monitor fallback along +d", recon, "fallback_step", fallback_step_ascending,
     [p_recon.test_monitor_with_a_diverging_inner_step_is_ista]),
    ("monitor fallback with half the threshold", recon, "fallback_step",
     fallback_step_half_threshold, [p_recon.test_monitor_with_a_diverging_inner_step_is_ista]),
]


@pytest.mark.parametrize("name,owner,attr,planted,pins", CASES, ids=[c[0] for c in CASES])
def test_pins_catch_the_planted_mistake(monkeypatch, name, owner, attr, planted, pins):
    # every pin passes on the oracle as it is (the pin modules run them too)
    monkeypatch.setattr(owner, attr, planted)
    for pin in pins:
        with pytest.raises(AssertionError):
            with np.errstate(all="ignore"):
                pin()
