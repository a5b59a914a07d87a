"""GPU parity of the db4 prox (Sec. 2.1, regularizer 2), the PCA basis and
the structured sketch (Sec. 2.3.2-2.3.3, Eq. 13) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import sketch as sk
from oracle import wavelet as wv
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu


def _cart_ctx(shape, C, levels=4):
    from paper_2305_06482_amd import Context
    return Context(shape, C, "cart", wav_levels=levels)


@pytest.mark.parametrize("shape,levels", [((128, 128), 4), ((320, 320), 4), ((48, 32), 3)])
def test_dwt_prox_2d(shape, levels):
    dev()
    case(f"dwt {shape} L={levels}")
    ctx = _cart_ctx(shape, 2, levels)
    x = rng_c(shape, 1)
    c = ctx.dwt(t(x))
    e = rel(h(c), wv.dwt(x, levels))
    assert e < 1e-5, e
    xi = ctx.idwt(c)
    e = rel(h(xi), x)
    assert e < 1e-5, e
    p = ctx.prox_l1wav(t(x), 0.3)
    e = rel(h(p), wv.prox_l1_wavelet(x, 0.3, levels))
    assert e < 1e-5, e
    ctx.close()


def test_dwt_prox_3d():
    dev()
    case("dwt 3d 48^3")
    from paper_2305_06482_amd import Context
    shape = (48, 48, 48)
    ctx = Context(shape, 4, "noncart", nsamp=10, wav_levels=4)
    x = rng_c(shape, 2)
    c = ctx.dwt(t(x))
    e = rel(h(c), wv.dwt(x, 4))
    assert e < 1e-5, e
    p = ctx.prox_l1wav(t(x), 0.5)
    e = rel(h(p), wv.prox_l1_wavelet(x, 0.5, 4))
    assert e < 1e-5, e
    ctx.close()


def test_coil_mix_matches_matmul():
    dev()
    case("coil_mix")
    shape, cin, cout = (40, 36), 13, 7
    ctx = _cart_ctx(shape, 2, 2)
    a = rng_c(shape + (cin,), 3)
    M = rng_c((cout, cin), 4)
    out = h(ctx.coil_mix(t(a), M))
    ref = a @ M.T
    e = rel(out, ref)
    assert e < 2e-6, e
    # +-1 entries (exact in bf16): only the data is split
    Ms = np.sign(np.random.default_rng(5).standard_normal((cout, cin)))
    out = h(ctx.coil_mix(t(a), Ms))
    e = rel(out, a @ Ms.T)
    assert e < 2e-6, e
    ctx.close()


@pytest.mark.parametrize("shape,C,V,S", [((128, 128), 8, 2, 2), ((64, 64), 12, 4, 3)])
def test_sketch_build_matches_oracle(shape, C, V, S):
    dev()
    case(f"sketch {shape} C={C} V={V} S={S}")
    x = synth.phantom(shape, 1)
    maps = synth.coil_maps(shape, C, 2)
    mask = synth.mask_1d_vd(shape[0], shape[1], 3, n_center=shape[0] // 8, accel=4)
    y = cart.forward(x, maps, mask) + synth.complex_noise(shape + (C,), 1e-3, 4) * mask[..., None]
    y = y.astype(np.complex64).astype(np.complex128)
    maps32 = maps.astype(np.complex64).astype(np.complex128)
    from paper_2305_06482_amd import Context
    import torch
    ctx = Context(shape, C, "cart")
    ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
    for tt in (1, 2, 7):
        sm, lam, U, sg = ctx.sketch_build(t(y), V, S, seed=77, t=tt)
        R = sk.covariance(y.reshape(-1, C))
        lam_r, U_r = sk.pca(R)
        assert np.max(np.abs(lam - lam_r)) < 1e-10 * lam_r[0]
        assert np.max(np.abs(U - U_r)) < 1e-8
        assert np.array_equal(sg, sk.rademacher(77, tt, S, C - V))
        ref, _ = sk.sketch_for_iteration(sk.virtual_maps(maps32, U_r), V, S, 77, tt)
        e = rel(h(sm), ref)
        assert e < 1e-5, e
    # V = C, S = 0 reduces to the virtual maps
    sm, _, U, _ = ctx.sketch_build(t(y), C, 0, seed=1, t=1)
    e = rel(h(sm), sk.virtual_maps(maps32, U))
    assert e < 1e-5, e
    ctx.close()
