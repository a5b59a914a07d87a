"""GPU parity at the workloads' own sizes, against the FP64 oracle.

* 2D Cartesian at clinical size (320^2, 32 coils, Poisson-disc mask R = 6,
  sketch 4 PCA + 4 Rademacher): Algorithm 1 after a fixed T x K, NRMSE
  <= 1e-3 (Sec. 2.3.4, Algorithm 1).
* The batched radial slices at the two ends of their size range: n = 384
  with 402 spokes and 32 coils (sketch 8 + 8), and n = 128 with 64 spokes
  and 8 coils (sketch 2 + 2): the operator to 1e-4 per apply and a short
  Algorithm 1 to NRMSE <= 1e-3 (radial slices, Sec. 3.2.1).
* Resuming Algorithm 1 at t0 = 6 from x^6 (b and the PCA basis reused)
  gives the uninterrupted 10-iteration result bit for bit: the inner FISTA
  restarts its momentum at every outer iteration and the sketch of outer
  iteration t depends only on (seed, t).

A fixed step alpha goes to both sides where the oracle's power iteration
would dominate the test time (FISTA converges for any alpha <= 1/L; parity
is checked iteration for iteration)."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import nufft
from oracle import recon as orecon
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu


def test_recon_cartesian_clinical_320():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    p = synth.make_cart_clinical()
    case("recon cart320 C=32 sketch 4+4 T=4 K=5")
    shape, C = p.shape, p.n_coils
    y = cart.forward(p.x_true, p.maps, p.mask) + p.noise.reshape(shape + (C,)) * p.mask[..., None]
    y = y.astype(np.complex64).astype(np.complex128)
    maps = p.maps.astype(np.complex64).astype(np.complex128)
    nf = lambda v, m: cart.normal(v, m, p.mask)
    b = cart.adjoint(y, maps, p.mask)
    T, K = 4, 5
    xr, alpha, _ = orecon.coil_sketch(nf, maps, y.reshape(-1, C), None, b,
                                      np.zeros(shape, complex), p.V, p.S, p.seed, T, K, p.lam)
    ctx = Context(shape, C, "cart")
    ctx.set_operator(t(maps), mask=t(p.mask, torch.uint8))
    res = ctx.recon_run(t(y), mode="sketch", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed,
                        step=alpha)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    assert res.n_full_applies == T and res.n_sketch_applies == T * K
    ctx.close()


@pytest.mark.parametrize("n,spokes,C,V", [(384, 402, 32, 8), (128, 64, 8, 2)])
def test_batched_slice_extremes(n, spokes, C, V):
    dev()
    from paper_2305_06482_amd import Context
    case(f"radial slice n={n} spokes={spokes} C={C} sketch {V}+{V}")
    p = synth.make_radial(n, spokes, C, V, V, seed_base=6000 + n)
    coords = p.coords.astype(np.float32).astype(np.float64)
    dcf = p.dcf.astype(np.float32).astype(np.float64)
    maps = p.maps.astype(np.complex64).astype(np.complex128)
    plan = nufft.Plan(p.shape, coords, dcf)
    ctx = Context(p.shape, C, "noncart", nsamp=coords.shape[0], wav_levels=4)
    mt = t(maps)
    ctx.set_operator(mt, coords=t(coords.astype(np.float32)), dcf=t(dcf.astype(np.float32)))
    # the operator, 4 of the coils (the oracle's NUFFT runs coil by coil)
    m4 = np.ascontiguousarray(maps[..., :4])
    x = synth.phantom(p.shape, 3) + 0.1 * rng_c(p.shape, 4)
    assert rel(h(ctx.sense_apply(t(m4), t(x))), plan.forward(x, m4)) < 1e-4
    assert rel(h(ctx.normal_apply(t(m4), t(x))), plan.normal(x, m4)) < 1e-4
    yy = rng_c((coords.shape[0], 4), 5)
    assert rel(h(ctx.sense_adjoint(t(m4), t(yy))), plan.adjoint(yy, m4)) < 1e-4
    # Algorithm 1, T = 1 outer iteration of K = 2
    y = plan.forward(p.x_true, maps) + p.noise * np.sqrt(dcf)[:, None]
    y = y.astype(np.complex64).astype(np.complex128)
    b = plan.adjoint(y, maps)
    alpha = 0.5
    xr, _, _ = orecon.coil_sketch(lambda v, m: plan.normal(v, m), maps, y, dcf, b,
                                  np.zeros(p.shape, complex), V, V, p.seed, 1, 2, p.lam,
                                  alpha=alpha)
    res = ctx.recon_run(t(y), mode="sketch", lam=p.lam, T=1, K=2, V=V, S=V, seed=p.seed,
                        step=alpha)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    ctx.close()


def test_resume_at_t0_is_bit_exact():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    p = synth.make_cart_small()
    case("resume cart128: 10 outer iterations vs 5 + 5")
    shape, C = p.shape, p.n_coils
    y = cart.forward(p.x_true, p.maps, p.mask) + p.noise.reshape(shape + (C,)) * p.mask[..., None]
    yt = t(y)
    maps = t(p.maps)
    ctx = Context(shape, C, "cart")
    ctx.set_operator(maps, mask=t(p.mask, torch.uint8))
    kw = dict(mode="sketch", lam=p.lam, K=5, V=p.V, S=p.S, seed=p.seed, step=0.4)
    full = ctx.recon_run(yt, T=10, **kw)
    xa = full.x.clone()
    first = ctx.recon_run(yt, T=5, **kw)
    second = ctx.recon_run(yt, T=5, t0=6, reuse_b=True, x=first.x.clone(), **kw)
    torch.cuda.synchronize()
    assert torch.equal(second.x, xa)
    ctx.close()
