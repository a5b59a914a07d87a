"""l1-TV reconstruction with PDHG (CG data consistency) on the GPU against the
FP64 oracle after a fixed number of iterations: the plain solver on
Cartesian, radial and 3D cones operators, and Algorithm 1 with PDHG inner
solves."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import nufft
from oracle import tv as otv
from tests.gpu_helpers import case, dev, h, rel, t

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _cart(n=64, C=8, seed=7100):
    import torch
    from paper_2305_06482_amd import Context
    shape = (n, n)
    maps = synth.coil_maps(shape, C, seed + 1).astype(np.complex64)
    mask = synth.mask_regular(n, n, accel=3, n_center=8)
    m64 = maps.astype(np.complex128)
    y = (cart.forward(synth.phantom(shape, seed), m64, mask) +
         synth.complex_noise(shape + (C,), 1e-3, seed + 2) * mask[..., None]).astype(np.complex64)
    ctx = Context(shape, C, "cart", wav_levels=2)
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    return ctx, shape, m64, mask, y


def test_pdhg_cartesian_matches_oracle():
    dev()
    case("TV PDHG, Cartesian 64x64, 8 coils")
    ctx, shape, maps, mask, y = _cart()
    lam, T, ncg = 2e-3, 30, 5
    r = ctx.recon_run(t(y), mode="full", reg="tv", lam=lam, T=T, n_cg=ncg)
    b = cart.adjoint(y.astype(np.complex128), maps, mask)
    ref = otv.pdhg_full(lambda v: cart.normal(v, maps, mask), b, np.zeros(shape, complex), lam,
                        T, ncg)
    e = rel(h(r.x), ref)
    assert e < TOL, e
    # each warm-started CG solve forms its residual with one more apply
    assert r.n_full_applies == T * (ncg + 1) and r.alpha == 0.0
    ctx.close()


@pytest.mark.parametrize("kind", ["radial", "cones"])
def test_pdhg_noncartesian_matches_oracle(kind):
    dev()
    from paper_2305_06482_amd import Context
    case(f"TV PDHG, {kind}")
    if kind == "radial":
        shape, C = (48, 48), 6
        coords = synth.radial_traj(48, 30)
        dcf = synth.radial_dcf(coords, 48)
    else:  # 3D: all three difference axes, partial tiles in the gridding
        shape, C = (16, 24, 24), 5
        coords = synth.cones_traj(shape, 240, 40, seed=5)
        dcf = synth.cones_dcf(coords, shape)
    c32, w32 = coords.astype(np.float32), dcf.astype(np.float32)
    maps = synth.coil_maps(shape, C, 7201).astype(np.complex64)
    m64 = maps.astype(np.complex128)
    plan = nufft.Plan(shape, c32.astype(np.float64), w32.astype(np.float64))
    y = (plan.forward(synth.phantom(shape, 7202), m64) +
         synth.complex_noise((coords.shape[0], C), 1e-3, 7203) * np.sqrt(w32)[:, None]
         ).astype(np.complex64)
    ctx = Context(shape, C, "noncart", nsamp=coords.shape[0], wav_levels=2)
    ctx.set_operator(t(maps), coords=t(c32), dcf=t(w32))
    lam, T, ncg = 2e-3, 15, 4
    r = ctx.recon_run(t(y), mode="full", reg="tv", lam=lam, T=T, n_cg=ncg)
    b = plan.adjoint(y.astype(np.complex128), m64)
    ref = otv.pdhg_full(lambda v: plan.normal(v, m64), b, np.zeros(shape, complex), lam, T, ncg)
    e = rel(h(r.x), ref)
    assert e < TOL, e
    ctx.close()


@pytest.mark.parametrize("V,S", [(3, 1), (2, 2)])
def test_pdhg_algorithm1_matches_oracle(V, S):
    dev()
    case(f"TV Algorithm 1, Cartesian 64x64, V={V} S={S}")
    ctx, shape, maps, mask, y = _cart(seed=7300)
    C = maps.shape[-1]
    lam, T, K, ncg, seed = 2e-3, 3, 10, 4, 41
    r = ctx.recon_run(t(y), mode="sketch", reg="tv", lam=lam, T=T, K=K, V=V, S=S, seed=seed,
                      n_cg=ncg)
    y64 = y.astype(np.complex128)
    b = cart.adjoint(y64, maps, mask)
    nfn = lambda v, m: cart.normal(v, m, mask)
    ref, _ = otv.pdhg_sketch(nfn, maps, y64.reshape(-1, C), None, b, np.zeros(shape, complex),
                             V, S, seed, T, K, lam, ncg)
    e = rel(h(r.x), ref)
    assert e < TOL, e
    assert r.n_full_applies == T and r.n_sketch_applies == T * (1 + K * (ncg + 1))
    ctx.close()
