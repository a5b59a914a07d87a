"""l2 (Tikhonov) reconstruction with conjugate gradients on the GPU against
the FP64 oracle: the plain solver (Cartesian and radial), Algorithm 1 with
CG inner solves, and the Monte-Carlo noise map of the linear reconstruction
against its closed form."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import l2 as ol2
from oracle import nufft
from tests.gpu_helpers import case, dev, h, rel, t

pytestmark = pytest.mark.gpu


def _cart(n=64, C=8, seed=6100, accel=3):
    import torch
    from paper_2305_06482_amd import Context
    shape = (n, n)
    x = synth.phantom(shape, seed)
    maps = synth.coil_maps(shape, C, seed + 1)
    mask = synth.mask_regular(n, n, accel=accel, n_center=8)
    y = cart.forward(x, maps, mask) + synth.complex_noise(shape + (C,), 1e-3, seed + 2) * \
        mask[..., None]
    y = y.astype(np.complex64)
    maps = maps.astype(np.complex64)
    ctx = Context(shape, C, "cart", wav_levels=2)
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    return ctx, shape, maps.astype(np.complex128), mask, y


def test_full_cg_cartesian_matches_oracle():
    dev()
    case("l2 full CG, Cartesian 64x64, 8 coils, regular R=3")
    ctx, shape, maps, mask, y = _cart()
    lam, T = 1e-2, 25
    r = ctx.recon_run(t(y), mode="full", reg="l2", lam=lam, T=T)
    y64 = y.astype(np.complex128)
    b = cart.adjoint(y64, maps, mask)
    ref = ol2.l2_full(lambda v: cart.normal(v, maps, mask), b, np.zeros(shape, complex), lam, T)
    e = rel(h(r.x), ref)
    assert e < 1e-4, e
    assert r.alpha == 0.0 and r.n_full_applies == T + 1 and r.n_prox == 0
    ctx.close()


def test_full_cg_radial_matches_oracle():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case("l2 full CG, radial 64, 8 coils")
    p = synth.make_radial(64, 48, 8, 3, 1, seed_base=6200)
    ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0], wav_levels=2)
    maps32 = p.maps.astype(np.complex64)
    dcf32 = p.dcf.astype(np.float32)
    c32 = p.coords.astype(np.float32)
    ctx.set_operator(t(maps32), coords=t(c32), dcf=t(dcf32))
    plan = nufft.Plan(p.shape, c32.astype(np.float64), dcf32.astype(np.float64))
    m64 = maps32.astype(np.complex128)
    y = (plan.forward(p.x_true, m64) + p.noise * np.sqrt(dcf32)[:, None]).astype(np.complex64)
    lam, T = 1e-2, 20
    r = ctx.recon_run(t(y), mode="full", reg="l2", lam=lam, T=T)
    b = plan.adjoint(y.astype(np.complex128), m64)
    ref = ol2.l2_full(lambda v: plan.normal(v, m64), b, np.zeros(p.shape, complex), lam, T)
    e = rel(h(r.x), ref)
    assert e < 1e-4, e
    ctx.close()


@pytest.mark.parametrize("V,S", [(3, 1), (2, 2)])
def test_sketched_l2_matches_oracle(V, S):
    dev()
    case(f"l2 Algorithm 1, Cartesian 64x64, 8 coils, V={V} S={S}")
    ctx, shape, maps, mask, y = _cart(seed=6300)
    C = maps.shape[-1]
    lam, T, K, seed = 1e-2, 4, 8, 31
    r = ctx.recon_run(t(y), mode="sketch", reg="l2", lam=lam, T=T, K=K, V=V, S=S, seed=seed)
    y64 = y.astype(np.complex128).reshape(-1, C)
    b = cart.adjoint(y64.reshape(shape + (C,)), maps, mask)
    nfn = lambda v, m: cart.normal(v, m, mask)
    ref, _ = ol2.l2_sketch(nfn, maps, y64, None, b, np.zeros(shape, complex), V, S, seed, T, K,
                           lam)
    e = rel(h(r.x), ref)
    assert e < 1e-3, e
    assert r.n_full_applies == T and r.n_sketch_applies == T * K
    ctx.close()


def test_sketched_l2_reaches_the_full_minimizer():
    dev()
    case("l2 Algorithm 1 converges to the full CG solution")
    ctx, shape, maps, mask, y = _cart(seed=6400)
    C = maps.shape[-1]
    lam = 1e-2
    yt = t(y)
    x_inf = ctx.recon_run(yt, mode="full", reg="l2", lam=lam, T=200).x
    # V = 5, S = 1 of 8 coils: the FP64 reference contracts by about 10x per
    # outer iteration here (to 1e-12 after 12); V = 3, S = 1 squeezes five
    # virtual coils into one and stalls near 1e-3, on both sides
    r = ctx.recon_run(yt, mode="sketch", reg="l2", lam=lam, T=12, K=30, V=5, S=1, seed=5,
                      x_ref=x_inf)
    assert r.dist[-1] < 1e-4, r.dist
    assert r.dist[-1] < 1e-2 * r.dist[0]
    ctx.close()


def test_monte_carlo_noise_map_matches_closed_form():
    """The noise map of the linear l2 reconstruction, estimated from 400
    reconstructions of pure white noise, against sqrt(diag(G G^H))."""
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case("l2 noise map by Monte Carlo, 16x16, 4 coils, regular R=2")
    n, C = 16, 4
    shape = (n, n)
    maps = synth.coil_maps(shape, C, 6501).astype(np.complex64)
    mask = synth.mask_regular(n, n, accel=2)
    lam = 5e-2
    A = cart.dense_matrix(maps.astype(np.complex128), mask)
    s_ref = ol2.noise_std(A, lam).reshape(shape)
    ctx = Context(shape, C, "cart", wav_levels=2)
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    gen = torch.Generator(device="cuda").manual_seed(7)
    m = t(mask, torch.float32)[..., None]
    acc = torch.zeros(shape, dtype=torch.float64, device="cuda")
    trials = 400
    for _ in range(trials):
        nz = torch.randn(shape + (C, 2), generator=gen, device="cuda") / np.sqrt(2.0)
        yk = torch.view_as_complex(nz.contiguous()) * m
        x = ctx.recon_run(yk.contiguous(), mode="full", reg="l2", lam=lam, T=60).x
        acc += x.abs().double() ** 2
    s_mc = (acc / trials).sqrt().cpu().numpy()
    ratio = s_mc / s_ref
    # sampling error of a standard deviation from 400 trials: about 3.5%
    assert abs(np.median(ratio) - 1) < 0.03, np.median(ratio)
    assert np.percentile(np.abs(ratio - 1), 95) < 0.1
    ctx.close()


def test_l2_rejects_learned_mode_and_unknown_regularizer():
    dev()
    from paper_2305_06482_amd import CNN, CSError
    case("l2: learned mode rejected")
    ctx, shape, maps, mask, y = _cart(n=32, seed=6600)
    net = CNN(seed=1)
    with pytest.raises(CSError):
        ctx.recon_run(t(y), mode="learned", reg="l2", T=1, K=2, V=2, S=2, cnn=net)
    net.close()
    ctx.close()
