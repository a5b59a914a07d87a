"""GPU parity of the non-Cartesian SENSE operator (Eqs. 1, 5; KB NUFFT)
against the FP64 oracle's NUFFT: relative L2 <= 1e-4 per apply."""
import numpy as np
import pytest

import synth
from oracle import nufft
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _setup(shape, coords, dcf, C, seed=2):
    from paper_2305_06482_amd import Context
    maps = synth.coil_maps(shape, C, seed)
    ctx = Context(shape, C, "noncart", nsamp=coords.shape[0], sigma=1.25,
                  wav_levels=2 if min(shape) < 48 else 4)
    ctx.set_operator(t(maps), coords=t(coords.astype(np.float32)),
                     dcf=t(dcf.astype(np.float32)))
    plan = nufft.Plan(shape, coords.astype(np.float32).astype(np.float64),
                      dcf.astype(np.float32).astype(np.float64))
    return ctx, maps, plan


def _check(ctx, maps, plan, shape, C, N, seed=0):
    x = synth.phantom(shape, 1) + 0.1 * rng_c(shape, seed + 9)
    mt = t(maps)
    y = ctx.sense_apply(mt, t(x))
    e = rel(h(y), plan.forward(x, maps))
    assert e < TOL, e
    yy = rng_c((N, C), seed + 4)
    xa = ctx.sense_adjoint(mt, t(yy))
    e = rel(h(xa), plan.adjoint(yy, maps))
    assert e < TOL, e
    n = ctx.normal_apply(mt, t(x))
    e = rel(h(n), plan.normal(x, maps))
    assert e < TOL, e
    lhs = np.vdot(h(y), yy)
    rhs = np.vdot(x, h(xa))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


@pytest.mark.parametrize("n,spokes,C", [(64, 24, 4), (48, 17, 3)])
def test_radial_2d(n, spokes, C):
    dev()
    case(f"radial n={n} spokes={spokes} C={C}")
    coords = synth.radial_traj(n, spokes)
    dcf = synth.radial_dcf(coords, n)
    ctx, maps, plan = _setup((n, n), coords, dcf, C)
    _check(ctx, maps, plan, (n, n), C, coords.shape[0])
    ctx.close()


@pytest.mark.parametrize("shape,nread,nsamp,C", [
    ((16, 24, 24), 120, 32, 5),
    ((48, 48, 48), 1125, 128, 12),
])
def test_cones_3d(shape, nread, nsamp, C):
    dev()
    case(f"cones {shape} C={C}")
    coords = synth.cones_traj(shape, nread, nsamp, seed=3)
    dcf = synth.cones_dcf(coords, shape)
    ctx, maps, plan = _setup(shape, coords, dcf, C)
    _check(ctx, maps, plan, shape, C, coords.shape[0])
    ctx.close()


def test_cones_full_coils_two_chunks():
    # 32 coils (two coil chunks of the gridding pipeline) on the 48^3 instance
    dev()
    case("cones 48^3 C=32")
    p = synth.make_cones_small()
    coords, dcf = p.coords, p.dcf
    ctx, maps, plan = _setup(p.shape, coords, dcf, 32, seed=3002)
    x = p.x_true
    n = ctx.normal_apply(t(maps), t(x))
    e = rel(h(n), plan.normal(x, maps))
    assert e < TOL, e
    ctx.close()


def test_normal_is_deterministic():
    dev()
    case("nufft determinism")
    shape = (24, 24, 24)
    coords = synth.cones_traj(shape, 300, 48, seed=4)
    dcf = synth.cones_dcf(coords, shape)
    ctx, maps, plan = _setup(shape, coords, dcf, 6)
    x = t(rng_c(shape, 3))
    a = h(ctx.normal_apply(t(maps), x))
    b = h(ctx.normal_apply(t(maps), x))
    assert np.array_equal(a, b)
    ctx.close()


@pytest.mark.parametrize("kind,C", [("radial", 3), ("radial", 16), ("tiny", 2), ("cones", 5),
                                    ("cones", 12), ("cones", 32)])
def test_interp_variants_agree(kind, C):
    """The global-memory gather (variant 0) and the LDS-tile interpolation
    (variants 1, 2, 3: coil groups of 8, 12, 4; 4: variant 3 with the tile
    interleaved as (re, im) pairs) against the oracle and
    against each other: same taps, same summation order.  Shapes with partial edge tiles (grid 30 = 3 x 8 + 6),
    odd coil counts (guarded group lanes), a grid shorter than the tile and
    two coil chunks."""
    dev()
    case(f"interp variants {kind} C={C}")
    if kind == "radial":
        shape = (40, 40)
        coords = synth.radial_traj(40, 21)
        dcf = synth.radial_dcf(coords, 40)
    elif kind == "tiny":  # grid 5 x 5: the halo'd tile wraps around it several times
        shape = (4, 4)
        coords = synth.radial_traj(4, 5)
        dcf = synth.radial_dcf(coords, 4)
    else:
        shape = (16, 24, 24)
        coords = synth.cones_traj(shape, 140, 40, seed=5)
        dcf = synth.cones_dcf(coords, shape)
    ctx, maps, plan = _setup(shape, coords, dcf, C, seed=7)
    x = synth.phantom(shape, 2) + 0.1 * rng_c(shape, 11)
    mt, xt = t(maps), t(x)
    out = {}
    for v in (0, 1, 2, 3, 4):
        ctx.set_interp_cfg(v)
        out[v] = (h(ctx.sense_apply(mt, xt)), h(ctx.normal_apply(mt, xt)))
    for v in (1, 2, 3, 4):
        assert rel(out[v][0], plan.forward(x, maps)) < TOL
        assert rel(out[v][1], plan.normal(x, maps)) < TOL
        for a, b in zip(out[0], out[v]):
            assert rel(b, a) < 1e-6
    ctx.close()


@pytest.mark.parametrize("kind,C", [("radial", 12), ("cones", 12), ("cones", 16), ("cones", 32),
                                    ("cones", 5), ("cart", 8)])
def test_paired_accesses_are_bit_identical(kind, C, monkeypatch):
    """The 16-byte coil-pair accesses of the grid FFT passes, the
    interpolation and the merge (the default) against one coil per access
    (CS_FFT_VEC=0, CS_FFT_VEC_IMG=0 and CS_GRID_VEC=0 when the context is
    made, with the image-prologue passes in whole-pixel panels,
    CS_FFT_PRO_COLS=0, and the coil sums by one thread per pixel,
    CS_FFT_SUM_ROWS=0): the same values move in the same order, so the
    forward, adjoint and normal applies agree bit for bit (odd coil counts
    take the one-coil path either way)."""
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case(f"paired accesses {kind} C={C}")
    if kind == "radial":
        shape = (40, 40)
        coords = synth.radial_traj(40, 21)
        dcf = synth.radial_dcf(coords, 40)
    elif kind == "cones":
        shape = (16, 24, 24)
        coords = synth.cones_traj(shape, 140, 40, seed=5)
        dcf = synth.cones_dcf(coords, shape)
    else:
        shape = (48, 40)
        mask = synth.mask_1d_vd(48, 40, 3, n_center=8, accel=2)
    maps = synth.coil_maps(shape, C, 7)
    x = synth.phantom(shape, 2) + 0.1 * rng_c(shape, 11)
    mt, xt = t(maps), t(x)
    outs = []
    knobs = ("CS_FFT_VEC", "CS_FFT_VEC_IMG", "CS_GRID_VEC", "CS_FFT_PRO_COLS", "CS_FFT_SUM_ROWS")
    for env in ({}, {k: "0" for k in knobs}):
        for k in knobs:
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        if kind == "cart":
            ctx = Context(shape, C, "cart", wav_levels=2)
            ctx.set_operator(mt, mask=t(mask, torch.uint8))
            yshape = shape + (C,)
        else:
            ctx = Context(shape, C, "noncart", nsamp=coords.shape[0], sigma=1.25, wav_levels=2)
            ctx.set_operator(mt, coords=t(coords.astype(np.float32)),
                             dcf=t(dcf.astype(np.float32)))
            yshape = (coords.shape[0], C)
        yt = t(rng_c(yshape, 4))
        outs.append((h(ctx.sense_apply(mt, xt)), h(ctx.sense_adjoint(mt, yt)),
                     h(ctx.normal_apply(mt, xt))))
        ctx.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
