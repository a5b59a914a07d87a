"""GPU parity of the Cartesian SENSE operator (Sec. 2.1, Eq. 2, F~ = U F~_u)
against the FP64 oracle: relative L2 <= 1e-4 per apply."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _ctx(shape, C, mask, maps):
    from paper_2305_06482_amd import Context
    ctx = Context(shape, C, "cart", wav_levels=2)
    ctx.set_operator(t(maps), mask=t(mask, __import__("torch").uint8))
    return ctx


@pytest.mark.parametrize("shape,C,kind", [
    ((128, 128), 8, "1d"),       # small Cartesian workload: 1D mask, fused y-only path
    ((64, 48), 5, "poisson"),    # ragged panel widths, odd coil count
    ((320, 320), 32, "poisson"), # clinical-size workload, two coil chunks
    ((60, 40), 3, "1d"),         # radix-3/5 lengths
])
def test_apply_adjoint_normal(shape, C, kind):
    dev()
    ny, nx = shape
    case(f"cart {shape} C={C} {kind}")
    maps = synth.coil_maps(shape, C, 2)
    if kind == "1d":
        mask = synth.mask_1d_vd(ny, nx, 3, n_center=min(24, ny // 4), accel=4)
    else:
        mask = synth.mask_poisson(ny, nx, 3, accel=6.0 if ny >= 128 else 3.0,
                                  calib=min(24, ny // 4))
    x = synth.phantom(shape, 1) + 0.1 * rng_c(shape, 9)
    ctx = _ctx(shape, C, mask, maps)
    mt = t(maps)
    y = ctx.sense_apply(mt, t(x))
    yr = cart.forward(x, maps, mask)
    e = rel(h(y), yr)
    assert e < TOL, e
    yy = rng_c(shape + (C,), 4) * mask[..., None]
    xa = ctx.sense_adjoint(mt, t(yy))
    e = rel(h(xa), cart.adjoint(yy, maps, mask))
    assert e < TOL, e
    n = ctx.normal_apply(mt, t(x))
    e = rel(h(n), cart.normal(x, maps, mask))
    assert e < TOL, e
    # adjointness on the GPU
    lhs = np.vdot(h(y), yy)
    rhs = np.vdot(x, h(xa))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)
    ctx.close()


def test_normal_is_deterministic():
    dev()
    case("cart determinism")
    shape, C = (96, 80), 6
    maps = synth.coil_maps(shape, C, 5)
    mask = synth.mask_poisson(96, 80, 6, accel=3.0, calib=16)
    ctx = _ctx(shape, C, mask, maps)
    x = t(rng_c(shape, 1))
    a = h(ctx.normal_apply(t(maps), x))
    b = h(ctx.normal_apply(t(maps), x))
    assert np.array_equal(a, b)
    ctx.close()
