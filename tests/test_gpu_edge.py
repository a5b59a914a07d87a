"""Degenerate and boundary cases of the operators on the GPU: an empty
trajectory, single samples on the exact -n/2 edge, one coil, empty and full
Cartesian masks (closed forms), and the 64-coil maximum of the sketch."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import nufft
from oracle import sketch as osk
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(32, 32), (16, 16, 16)])
def test_empty_trajectory_is_the_zero_operator(shape):
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case(f"empty trajectory {shape}")
    nd = len(shape)
    ctx = Context(shape, 3, "noncart", nsamp=0, wav_levels=2)
    maps = t(rng_c(shape + (3,), 1).astype(np.complex64))
    ctx.set_operator(maps, coords=torch.zeros((0, nd), dtype=torch.float32, device="cuda"),
                     dcf=torch.zeros((0,), dtype=torch.float32, device="cuda"))
    x = t(rng_c(shape, 2).astype(np.complex64))
    assert float(ctx.normal_apply(maps, x).abs().max()) == 0.0
    y = ctx.sense_apply(maps, x)
    assert y.shape == (0, 3)
    assert float(ctx.sense_adjoint(maps, y).abs().max()) == 0.0
    ctx.close()


@pytest.mark.parametrize("shape", [(32, 32), (16, 16, 16)])
def test_single_samples_on_the_edge_and_one_coil(shape):
    dev()
    from paper_2305_06482_amd import Context
    nd = len(shape)
    n = np.array(shape[::-1], dtype=np.float64)  # coordinate columns x, y(, z)
    coords = np.stack([-n / 2, np.zeros(nd), n / 2 - 1e-3, -n / 2 + 0.5], 0)  # edges and DC
    dcf = np.array([0.7, 1.0, 1.3, 0.2])
    for C in (1, 3):
        case(f"edge samples {shape}, {C} coil(s)")
        maps = rng_c(shape + (C,), 3).astype(np.complex64)
        x = rng_c(shape, 4).astype(np.complex64)
        ctx = Context(shape, C, "noncart", nsamp=coords.shape[0], wav_levels=2)
        ctx.set_operator(t(maps), coords=t(coords.astype(np.float32)),
                         dcf=t(dcf.astype(np.float32)))
        plan = nufft.Plan(shape, coords.astype(np.float32).astype(np.float64),
                          dcf.astype(np.float32).astype(np.float64))
        m64, x64 = maps.astype(np.complex128), x.astype(np.complex128)
        assert rel(h(ctx.sense_apply(t(maps), t(x))), plan.forward(x64, m64)) < 1e-4
        assert rel(h(ctx.normal_apply(t(maps), t(x))), plan.normal(x64, m64)) < 1e-4
        yy = rng_c((coords.shape[0], C), 5).astype(np.complex64)
        assert rel(h(ctx.sense_adjoint(t(maps), t(yy))),
                   plan.adjoint(yy.astype(np.complex128), m64)) < 1e-4
        ctx.close()


def test_cartesian_empty_and_full_masks():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    shape, C = (48, 40), 5
    maps = rng_c(shape + (C,), 6).astype(np.complex64)
    x = rng_c(shape, 7).astype(np.complex64)
    for name, mask in (("empty", np.zeros(shape, np.uint8)), ("full", np.ones(shape, np.uint8))):
        case(f"Cartesian {name} mask")
        ctx = Context(shape, C, "cart", wav_levels=2)
        ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
        got = h(ctx.normal_apply(t(maps), t(x)))
        if name == "empty":
            assert np.abs(got).max() == 0.0
        else:
            # U^H U = I: the normal operator is x times the coil sum of |c|^2
            ref = x.astype(np.complex128) * np.sum(np.abs(maps.astype(np.complex128)) ** 2, -1)
            assert rel(got, ref) < 1e-5
            assert rel(got, cart.normal(x.astype(np.complex128), maps.astype(np.complex128),
                                        mask)) < 1e-5
        ctx.close()


def test_sketch_at_the_64_coil_maximum():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case("sketch_build with 64 coils (the maximum)")
    shape, C, V, S = (32, 32), 64, 6, 6
    x = synth.phantom(shape, 7003)
    maps = synth.coil_maps(shape, C, 7001)
    mask = synth.mask_1d_vd(32, 32, 7002, n_center=8, accel=2)
    y = cart.forward(x, maps, mask) + synth.complex_noise(shape + (C,), 1e-2, 7004) * mask[..., None]
    y = y.astype(np.complex64).astype(np.complex128)
    maps32 = maps.astype(np.complex64).astype(np.complex128)
    ctx = Context(shape, C, "cart", wav_levels=2)
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    sm, lam, U, sg = ctx.sketch_build(t(y), V, S, seed=9, t=1)
    lam_r, U_r = osk.pca(osk.covariance(y.reshape(-1, C)))
    # the smallest relative eigenvalue gap here is about 1e-5, so FP64
    # eigenvectors agree to ~1e-11
    assert np.max(np.abs(lam - lam_r)) < 1e-10 * lam_r[0]
    assert np.max(np.abs(U - U_r)) < 1e-8
    assert np.array_equal(sg, osk.rademacher(9, 1, S, C - V))
    ref, _ = osk.sketch_for_iteration(osk.virtual_maps(maps32, U_r), V, S, 9, 1)
    e = rel(h(sm), ref)
    assert e < 1e-5, e
    ctx.close()


def test_coil_count_beyond_the_maximum_is_rejected():
    dev()
    from paper_2305_06482_amd import Context, CSError
    case("65 coils: rejected at create")
    with pytest.raises(CSError):
        Context((32, 32), 65, "cart")
