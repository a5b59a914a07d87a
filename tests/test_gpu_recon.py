"""GPU reconstruction (Algorithm 1 with FISTA inner solves, and plain FISTA)
against the FP64 oracle after a fixed iteration count: NRMSE <= 1e-3.  The
oracle's step size is passed to both sides; the GPU power iteration is
checked separately against the oracle's."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import nufft
from oracle import recon as orecon
from tests.gpu_helpers import case, dev, h, rel, t

pytestmark = pytest.mark.gpu


def _cart_problem(p):
    shape, C = p.shape, p.n_coils
    y = cart.forward(p.x_true, p.maps, p.mask) + p.noise.reshape(shape + (C,)) * p.mask[..., None]
    y = y.astype(np.complex64).astype(np.complex128)
    maps = p.maps.astype(np.complex64).astype(np.complex128)
    return y, maps


def test_recon_small_cartesian_sketch_and_full():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    p = synth.make_cart_small()
    case("recon cart128")
    y, maps = _cart_problem(p)
    C = p.n_coils
    nf = lambda v, m: cart.normal(v, m, p.mask)
    b = cart.adjoint(y, maps, p.mask)
    T, K = 6, 5
    xr, alpha, st = orecon.coil_sketch(nf, maps, y.reshape(-1, C), None, b,
                                       np.zeros(p.shape, complex), p.V, p.S, p.seed, T, K, p.lam)
    ctx = Context(p.shape, C, "cart")
    ctx.set_operator(t(maps), mask=t(p.mask, torch.uint8))
    yt = t(y)
    res = ctx.recon_run(yt, mode="sketch", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed,
                        step=alpha)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    assert res.n_full_applies == T and res.n_sketch_applies == T * K
    # power iteration on the first subproblem
    L_gpu = ctx.power_iteration(ctx.sketch_build(yt, p.V, p.S, p.seed, 1)[0])
    assert abs(L_gpu - 1.0 / alpha) < 1e-4 / alpha
    # plain FISTA
    xf = orecon.fista_full(lambda v: nf(v, maps), b, np.zeros(p.shape, complex), alpha, p.lam, 12)
    resf = ctx.recon_run(yt, mode="full", lam=p.lam, T=12, step=alpha, reuse_b=True)
    e = orecon.nrmse(h(resf.x), xf)
    assert e < 1e-3, e
    ctx.close()


def test_recon_cones_48():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    p = synth.make_cones_small()
    case("recon cones48")
    C = p.n_coils
    coords = p.coords.astype(np.float32).astype(np.float64)
    dcf = p.dcf.astype(np.float32).astype(np.float64)
    plan = nufft.Plan(p.shape, coords, dcf)
    maps = p.maps.astype(np.complex64).astype(np.complex128)
    y = plan.forward(p.x_true, maps) + p.noise * np.sqrt(dcf)[:, None]
    y = y.astype(np.complex64).astype(np.complex128)
    b = plan.adjoint(y, maps)
    T, K = 2, 3
    xr, alpha, st = orecon.coil_sketch(lambda v, m: plan.normal(v, m), maps, y, dcf, b,
                                       np.zeros(p.shape, complex), p.V, p.S, p.seed, T, K, p.lam)
    ctx = Context(p.shape, C, "noncart", nsamp=coords.shape[0], wav_levels=4)
    ctx.set_operator(t(maps), coords=t(coords.astype(np.float32)), dcf=t(dcf.astype(np.float32)))
    res = ctx.recon_run(t(y), mode="sketch", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed,
                        step=alpha)
    e = orecon.nrmse(h(res.x), xr)
    assert e < 1e-3, e
    ctx.close()


def test_recon_monitor_cartesian():
    # objective monitor: F(x^t) against the oracle's F of its own iterates
    # (relative 1e-3), no fallback and no change to x on a converging run;
    # with the inner step forced 30x too large from the host every outer
    # iterate is replaced by the full-coil proximal-gradient step, matching
    # the oracle's monitored run (NRMSE <= 1e-3) with a non-increasing F
    dev()
    import torch
    from paper_2305_06482_amd import CSError, Context
    p = synth.make_cart_small()
    case("recon monitor cart128")
    y, maps = _cart_problem(p)
    C = p.n_coils
    yr = y.reshape(-1, C)
    nf = lambda v, m: cart.normal(v, m, p.mask)
    fwd = lambda v, m: cart.forward(v, m, p.mask).reshape(-1, m.shape[-1])
    b = cart.adjoint(y, maps, p.mask)
    T, K = 4, 5
    x0 = np.zeros(p.shape, complex)
    _, alpha, _ = orecon.coil_sketch(nf, maps, yr, None, b, x0, p.V, p.S, p.seed, 0, K, p.lam)
    ctx = Context(p.shape, C, "cart")
    ctx.set_operator(t(maps), mask=t(p.mask, torch.uint8))
    yt = t(y)
    kw = dict(mode="sketch", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed)
    plain = ctx.recon_run(yt, step=alpha, **kw)
    for scale, fallbacks in ((1.0, 0), (30.0, T)):
        case(f"recon monitor cart128 step x{scale}")
        xm, _, F0, F, fell = orecon.coil_sketch_monitored(
            nf, fwd, maps, yr, None, b, x0, p.V, p.S, p.seed, T, K, p.lam, 0.0,
            alpha=scale * alpha)
        assert sum(fell) == fallbacks
        res = ctx.recon_run(yt, step=scale * alpha, monitor=True, mon_tol=0.0, reuse_b=True, **kw)
        assert res.n_fallbacks == fallbacks
        assert res.n_full_applies == T + 1 + (fallbacks + 31 if fallbacks else 0)
        assert abs(res.objective0 - F0) <= 1e-6 * F0
        for got, want in zip(res.objective, F):
            assert abs(got - want) <= 1e-3 * want, (got, want)
        e = orecon.nrmse(h(res.x), xm)
        assert e < 1e-3, e
        if fallbacks == 0:
            assert torch.equal(res.x, plain.x)
        else:
            seq = [res.objective0] + res.objective
            assert all(seq[i + 1] <= seq[i] * (1 + 1e-5) for i in range(T)), seq
    with pytest.raises(CSError, match="monitor"):
        ctx.recon_run(yt, mode="full", lam=p.lam, T=2, step=alpha, monitor=True)
    with pytest.raises(CSError, match="mon_tol"):
        ctx.recon_run(yt, step=alpha, monitor=True, mon_tol=-1.0, **kw)
    ctx.close()
