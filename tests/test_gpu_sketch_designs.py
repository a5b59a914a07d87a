"""Sketch designs of Sec. 3.2 on the GPU against the FP64 oracle: Gaussian
entries (sketched maps and Algorithm 1), the S = 0 design (coil compression
inside the subproblem), and the divergence of S = 0 where S >= 1 converges."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import l2 as ol2
from oracle import recon as orecon
from oracle import sketch as sk
from tests.gpu_helpers import case, dev, h, rel, t

pytestmark = pytest.mark.gpu


def _sketch_case(shape=(64, 64), C=12):
    import torch
    from paper_2305_06482_amd import Context
    x = synth.phantom(shape, 1)
    maps = synth.coil_maps(shape, C, 2)
    mask = synth.mask_1d_vd(shape[0], shape[1], 3, n_center=8, accel=4)
    y = cart.forward(x, maps, mask) + synth.complex_noise(shape + (C,), 1e-3, 4) * mask[..., None]
    y = y.astype(np.complex64).astype(np.complex128)
    maps32 = maps.astype(np.complex64).astype(np.complex128)
    ctx = Context(shape, C, "cart")
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    return ctx, y, maps32, mask


@pytest.mark.parametrize("V,S", [(4, 3), (0, 5), (6, 0)])
def test_gaussian_and_s0_sketched_maps_match_oracle(V, S):
    dev()
    case(f"Gaussian / S=0 sketched maps V={V} S={S}")
    ctx, y, maps32, mask = _sketch_case()
    C = maps32.shape[-1]
    ctx.set_sketch_dist("gaussian")
    _, U_r = sk.pca(sk.covariance(y.reshape(-1, C)))
    vm = sk.virtual_maps(maps32, U_r)
    for tt in (1, 5):
        sm, lam, U, _ = ctx.sketch_build(t(y), V, S, seed=91, t=tt)
        ref, _ = sk.sketch_for_iteration(vm, V, S, 91, tt, "gaussian")
        e = rel(h(sm), ref)
        assert e < 1e-5, (tt, e)
    # back to Rademacher on the same context
    ctx.set_sketch_dist("rademacher")
    if S > 0:
        sm, _, _, sg = ctx.sketch_build(t(y), V, S, seed=91, t=2)
        assert np.array_equal(sg, sk.rademacher(91, 2, S, C - V))
        ref, _ = sk.sketch_for_iteration(vm, V, S, 91, 2)
        assert rel(h(sm), ref) < 1e-5
    ctx.close()


def test_gaussian_algorithm1_matches_oracle():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case("Algorithm 1 with Gaussian sketches, cart128")
    p = synth.make_cart_small()
    C = p.n_coils
    y = cart.forward(p.x_true, p.maps, p.mask) + p.noise.reshape(p.shape + (C,)) * \
        p.mask[..., None]
    y = y.astype(np.complex64).astype(np.complex128)
    maps = p.maps.astype(np.complex64).astype(np.complex128)
    nf = lambda v, m: cart.normal(v, m, p.mask)
    b = cart.adjoint(y, maps, p.mask)
    T, K = 5, 5
    xr, alpha, _ = orecon.coil_sketch(nf, maps, y.reshape(-1, C), None, b,
                                      np.zeros(p.shape, complex), 3, 1, p.seed, T, K, p.lam,
                                      dist="gaussian")
    ctx = Context(p.shape, C, "cart")
    ctx.set_operator(t(maps), mask=t(p.mask, torch.uint8))
    ctx.set_sketch_dist("gaussian")
    res = ctx.recon_run(t(y), mode="sketch", lam=p.lam, T=T, K=K, V=3, S=1, seed=p.seed,
                        step=alpha)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    ctx.close()


def test_s0_diverges_where_s1_converges_on_gpu():
    """The oracle pin's problem (l2, C^ = 4 of 8 coils): S = 0 moves away from
    the minimizer while V = 3, S = 1 converges, with either distribution; the
    GPU follows the oracle's outer iterations."""
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case("S = 0 divergence vs S = 1 convergence (l2)")
    shape, C, lam = (32, 32), 8, 1e-2
    x = synth.phantom(shape, 21)
    maps = synth.coil_maps(shape, C, 22).astype(np.complex64)
    mask = synth.mask_1d_vd(32, 32, 23, n_center=6, accel=2)
    m64 = maps.astype(np.complex128)
    y = (cart.forward(x, m64, mask) + 1e-3 * synth.complex_noise(shape + (C,), 1.0, 24) *
         mask[..., None]).astype(np.complex64)
    ctx = Context(shape, C, "cart", wav_levels=2)
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    yt = t(y)
    x_inf = ctx.recon_run(yt, mode="full", reg="l2", lam=lam, T=300).x
    y64 = y.astype(np.complex128)
    b = cart.adjoint(y64, m64, mask)
    nfn = lambda v, mm: cart.normal(v, mm, mask)
    # the oracle measures against its own FP64 minimizer
    ref_inf = ol2.l2_full(lambda v: cart.normal(v, m64, mask), b, np.zeros(shape, complex), lam,
                          300)
    for V, S, dist in ((4, 0, "rademacher"), (3, 1, "rademacher"), (3, 1, "gaussian")):
        ctx.set_sketch_dist(dist)
        r = ctx.recon_run(yt, mode="sketch", reg="l2", lam=lam, T=15, K=50, V=V, S=S, seed=3,
                          x_ref=x_inf)
        ref_d = []
        ol2.l2_sketch(nfn, m64, y64.reshape(-1, C), None, b, np.zeros(shape, complex), V, S, 3,
                      15, 50, lam, dist=dist,
                      callback=lambda tt, xx: ref_d.append(
                          np.linalg.norm(xx - ref_inf) / np.linalg.norm(ref_inf)))
        d = np.array(r.dist)
        # the same trajectory as the FP64 reference, to single-precision accuracy
        assert np.max(np.abs(d - np.array(ref_d)) / np.maximum(np.array(ref_d), 1e-5)) < 0.05, \
            (V, S, dist, d, ref_d)
        if S == 0:
            assert d[-1] > 3 * d.min(), d
        else:
            assert d[-1] < 1e-3, d
    ctx.close()


@pytest.mark.parametrize("kind", ["cart", "radial"])
def test_classical_init_matches_oracle(kind):
    """Alg. 1 with the classical-sketch initialisation (sketched data
    S~^0 U^H y, mixed on MFMA over the N data rows) against the oracle."""
    dev()
    import torch
    from paper_2305_06482_amd import Context
    from oracle import nufft
    case(f"classical-sketch initialisation, {kind}")
    T, K, K0 = 3, 5, 10
    if kind == "cart":
        p = synth.make_cart_small()
        C = p.n_coils
        y = cart.forward(p.x_true, p.maps, p.mask) + p.noise.reshape(p.shape + (C,)) * \
            p.mask[..., None]
        y = y.astype(np.complex64).astype(np.complex128)
        maps = p.maps.astype(np.complex64).astype(np.complex128)
        nf = lambda v, m: cart.normal(v, m, p.mask)
        af = lambda yy, m: cart.adjoint(yy.reshape(p.shape + (m.shape[-1],)), m, p.mask)
        b = cart.adjoint(y, maps, p.mask)
        ctx = Context(p.shape, C, "cart")
        ctx.set_operator(t(maps), mask=t(p.mask, torch.uint8))
        y2, dcf, yt = y.reshape(-1, C), None, t(y)
    else:  # N = 6144 samples on a 64 x 64 image: rows != pixels
        p = synth.make_radial(64, 48, 8, 2, 2, seed_base=7400)
        C = p.n_coils
        c32, w32 = p.coords.astype(np.float32), p.dcf.astype(np.float32)
        maps = p.maps.astype(np.complex64).astype(np.complex128)
        plan = nufft.Plan(p.shape, c32.astype(np.float64), w32.astype(np.float64))
        y2 = (plan.forward(p.x_true, maps) + p.noise * np.sqrt(w32)[:, None]
              ).astype(np.complex64).astype(np.complex128)
        nf = lambda v, m: plan.normal(v, m)
        af = lambda yy, m: plan.adjoint(yy, m)
        b = plan.adjoint(y2, maps)
        dcf = w32.astype(np.float64)
        ctx = Context(p.shape, C, "noncart", nsamp=c32.shape[0], wav_levels=4)
        ctx.set_operator(t(maps.astype(np.complex64)), coords=t(c32), dcf=t(w32))
        yt = t(y2)
    xr, alpha, _ = orecon.coil_sketch(nf, maps, y2, dcf, b, np.zeros(p.shape, complex), p.V,
                                      p.S, p.seed, T, K, p.lam, init_iters=K0,
                                      adjoint_maps_fn=af)
    res = ctx.recon_run(yt, mode="sketch", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed,
                        step=alpha, init_iters=K0)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    assert res.n_sketch_applies == K0 + T * K
    ctx.close()


@pytest.mark.parametrize("kind", ["cart", "radial"])
def test_initial_compression_matches_oracle(kind):
    """Alg. 1 after compressing to the first C0 = 6 of 8 virtual coils (model
    and data), against the oracle."""
    dev()
    import torch
    from paper_2305_06482_amd import Context
    from oracle import nufft
    case(f"initial coil compression C0=6, {kind}")
    T, K, C0, V, S = 3, 5, 6, 3, 1
    if kind == "cart":
        p = synth.make_cart_small()
        C = p.n_coils
        y = cart.forward(p.x_true, p.maps, p.mask) + p.noise.reshape(p.shape + (C,)) * \
            p.mask[..., None]
        y = y.astype(np.complex64).astype(np.complex128)
        maps = p.maps.astype(np.complex64).astype(np.complex128)
        nf = lambda v, m: cart.normal(v, m, p.mask)
        af = lambda yy, m: cart.adjoint(yy.reshape(p.shape + (m.shape[-1],)), m, p.mask)
        ctx = Context(p.shape, C, "cart")
        ctx.set_operator(t(maps), mask=t(p.mask, torch.uint8))
        y2, dcf, yt = y.reshape(-1, C), None, t(y)
    else:
        p = synth.make_radial(64, 48, 8, 2, 2, seed_base=7500)
        C = p.n_coils
        c32, w32 = p.coords.astype(np.float32), p.dcf.astype(np.float32)
        maps = p.maps.astype(np.complex64).astype(np.complex128)
        plan = nufft.Plan(p.shape, c32.astype(np.float64), w32.astype(np.float64))
        y2 = (plan.forward(p.x_true, maps) + p.noise * np.sqrt(w32)[:, None]
              ).astype(np.complex64).astype(np.complex128)
        nf = lambda v, m: plan.normal(v, m)
        af = lambda yy, m: plan.adjoint(yy, m)
        dcf = w32.astype(np.float64)
        ctx = Context(p.shape, C, "noncart", nsamp=c32.shape[0], wav_levels=4)
        ctx.set_operator(t(maps.astype(np.complex64)), coords=t(c32), dcf=t(w32))
        yt = t(y2)
    xr, alpha, _ = orecon.coil_sketch_compressed(nf, af, maps, y2, dcf,
                                                 np.zeros(p.shape, complex), C0, V, S, p.seed,
                                                 T, K, p.lam)
    res = ctx.recon_run(yt, mode="sketch", lam=p.lam, T=T, K=K, V=V, S=S, seed=p.seed,
                        step=alpha, C0=C0)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    # the next uncompressed call recomputes b = A^H y for all coils
    full = ctx.recon_run(yt, mode="sketch", lam=p.lam, T=1, K=K, V=V, S=S, seed=p.seed,
                         step=alpha, reuse_b=True)
    b = af(y2, maps)
    xr1, _, _ = orecon.coil_sketch(nf, maps, y2, dcf, b, np.zeros(p.shape, complex), V, S,
                                   p.seed, 1, K, p.lam, alpha=alpha)
    assert orecon.nrmse(h(full.x), xr1) < 1e-3
    ctx.close()
