"""Parity at the full 3D cones size (192x192x128 image, 18000 x 512 samples,
grid 240x240x160), in the launch configuration the benchmark uses.

The oracle's full-size NUFFT is affordable for one coil, so the one-coil
normal apply and forward operator are compared element by element; the
sketched 12-coil apply is checked through properties that hold at any size
(coil linearity against the one-coil applies, Hermitian positive
semi-definiteness, adjointness of the forward/adjoint pair)."""
import numpy as np
import pytest

import synth
from oracle import nufft
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu

SHAPE = (128, 192, 192)


@pytest.fixture(scope="module")
def full():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    coords = synth.cones_traj(SHAPE, 18000, 512, seed=3003)
    dcf = synth.cones_dcf(coords, SHAPE)
    maps = synth.coil_maps(SHAPE, 12, 3002).astype(np.complex64)
    x = synth.phantom(SHAPE, 3001).astype(np.complex64)
    ctx = Context(SHAPE, 12, "noncart", nsamp=coords.shape[0], wav_levels=4)
    ctx.set_operator(t(maps), coords=t(coords.astype(np.float32)),
                     dcf=t(dcf.astype(np.float32)))
    plan = nufft.Plan(SHAPE, coords.astype(np.float32).astype(np.float64),
                      dcf.astype(np.float32).astype(np.float64))
    yield ctx, plan, maps, x, coords
    ctx.close()


def test_one_coil_normal_full_size(full):
    ctx, plan, maps, x, coords = full
    case("full-size one-coil normal")
    m1 = np.ascontiguousarray(maps[..., :1])
    got = h(ctx.normal_apply(t(m1), t(x)))
    ref = plan.normal(x.astype(np.complex128), m1.astype(np.complex128))
    e = rel(got, ref)
    assert e < 1e-4, e


def test_one_coil_forward_sampled(full):
    ctx, plan, maps, x, coords = full
    case("full-size one-coil forward, sampled outputs")
    m1 = np.ascontiguousarray(maps[..., :1])
    got = h(ctx.sense_apply(t(m1), t(x)))[:, 0]
    ref = plan.forward(x.astype(np.complex128), m1.astype(np.complex128))[:, 0]
    idx = np.random.default_rng(0).choice(coords.shape[0], 20000, replace=False)
    e = rel(got[idx], ref[idx])
    assert e < 1e-4, e


def test_sketched_apply_properties(full):
    ctx, plan, maps, x, coords = full
    case("full-size 12-coil normal: coil linearity, PSD, adjointness")
    mt = t(maps)
    n12 = h(ctx.normal_apply(mt, t(x)))
    acc = np.zeros_like(n12)
    for j in range(12):
        acc += h(ctx.normal_apply(t(np.ascontiguousarray(maps[..., j:j + 1])), t(x)))
    e = rel(n12, acc)
    assert e < 1e-5, e
    q = np.vdot(x, n12)
    assert q.real > 0 and abs(q.imag) < 1e-5 * abs(q)
    y = h(ctx.sense_apply(mt, t(x)))
    yy = rng_c(y.shape, 5).astype(np.complex64)
    xa = h(ctx.sense_adjoint(mt, t(yy)))
    lhs, rhs = np.vdot(y, yy), np.vdot(x, xa)
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)
