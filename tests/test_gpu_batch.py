"""Batched slices (independent 2D radial reconstructions of uneven size, coil
count and sketch size, each on its own context and stream) and the
spreading-shape autotuner.

* The graph path (inner iterations captured once, replayed every outer
  iteration with the eager full-gradient and sketch work in between) equals
  the eager path bit for bit after 1, 2 and 3 outer iterations.
* The batch equals per-slice recon_run bit for bit (same kernels, same order).
* One slice matches the FP64 oracle's Algorithm 1 to NRMSE <= 1e-3.
* Every spreading shape gives bit-identical normal applies."""
import numpy as np
import pytest

import synth
from oracle import nufft
from oracle import recon as orecon
from tests.gpu_helpers import case, dev, h, t

pytestmark = pytest.mark.gpu

SPECS = [  # n, spokes, coils, V, S
    (48, 40, 8, 2, 2),
    (64, 57, 12, 3, 3),
    (80, 33, 9, 2, 2),
    (64, 71, 16, 4, 4),
    (96, 48, 10, 3, 3),
]
LAM, K = 1e-3, 4


def _slices(torch):
    from paper_2305_06482_amd import Context
    out = []
    for i, (n, spokes, C, V, S) in enumerate(SPECS):
        p = synth.make_radial(n, spokes, C, V, S, seed_base=5000 + 10 * i)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ctx = Context(p.shape, C, "noncart", nsamp=p.coords.shape[0], wav_levels=4)
            maps = t(p.maps.astype(np.complex64))
            dcf = t(p.dcf.astype(np.float32))
            ctx.set_operator(maps, coords=t(p.coords.astype(np.float32)), dcf=dcf)
            y = ctx.sense_apply(maps, t(p.x_true.astype(np.complex64)))
            y += t(p.noise.astype(np.complex64)) * dcf.sqrt()[:, None].to(torch.complex64)
        torch.cuda.synchronize()
        out.append((p, ctx, maps, y))
    return out


@pytest.fixture(scope="module")
def batch():
    dev()
    import torch
    sl = _slices(torch)
    yield torch, sl
    for _, ctx, _, _ in sl:
        ctx.close()


def _run(torch, sl, T, use_graph, step=None):
    from paper_2305_06482_amd import Batch
    xs = [torch.zeros(p.shape, dtype=torch.complex64, device="cuda") for p, *_ in sl]
    torch.cuda.synchronize()
    b = Batch([ctx for _, ctx, _, _ in sl])
    st = b.recon([y for *_, y in sl], xs, LAM, T, K, [p.V for p, *_ in sl],
                 [p.S for p, *_ in sl], [p.seed for p, *_ in sl], step=step,
                 use_graph=use_graph)
    b.close()
    return xs, st


def test_graph_replays_match_eager(batch):
    torch, sl = batch
    for T in (1, 2, 3):
        case(f"batch of {len(sl)} radial slices, T={T}: graph vs eager")
        xe, _ = _run(torch, sl, T, False)
        xg, st = _run(torch, sl, T, True)
        assert st[0]["graph_replays"] == T and st[0]["graph_nodes"] > 0
        for i, (a, b) in enumerate(zip(xe, xg)):
            assert torch.equal(a, b), (T, i)


def test_batch_matches_single_slice_runs(batch):
    torch, sl = batch
    case("batch vs per-slice recon_run")
    xb, st = _run(torch, sl, 2, True)
    for i, (p, ctx, maps, y) in enumerate(sl):
        with torch.cuda.stream(ctx.stream):
            r = ctx.recon_run(y, mode="sketch", lam=LAM, T=2, K=K, V=p.V, S=p.S, seed=p.seed,
                              step=0.0)
        torch.cuda.synchronize()
        assert abs(r.alpha - st[i]["alpha"]) <= 1e-12 * r.alpha, i
        assert torch.equal(r.x, xb[i]), i


def test_batch_slice_matches_oracle(batch):
    torch, sl = batch
    p, ctx, maps, y = sl[0]
    case("batch slice 0 vs FP64 oracle Algorithm 1")
    C = p.n_coils
    coords = p.coords.astype(np.float32).astype(np.float64)
    dcf = p.dcf.astype(np.float32).astype(np.float64)
    plan = nufft.Plan(p.shape, coords, dcf)
    maps64 = p.maps.astype(np.complex64).astype(np.complex128)
    y64 = h(y).astype(np.complex128)
    b = plan.adjoint(y64, maps64)
    T = 3
    xr, alpha, _ = orecon.coil_sketch(lambda v, m: plan.normal(v, m), maps64, y64, dcf, b,
                                      np.zeros(p.shape, complex), p.V, p.S, p.seed, T, K, LAM)
    steps = [alpha] + [0.0] * (len(sl) - 1)
    xb, _ = _run(torch, sl, T, True, step=steps)
    e = orecon.nrmse(h(xb[0]), xr)
    assert e < 1e-3, e


def test_spread_shapes_identical_and_autotune():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    from paper_2305_06482_amd.binding import SPREAD_NCFG
    for name, p in (("radial 64", synth.make_radial(64, 40, 12, 3, 3, seed_base=5100)),
                    ("cones 48^3", synth.make_cones_small())):
        case(f"spreading shapes, {name}")
        C = min(p.n_coils, 12)
        ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0],
                      wav_levels=3 if len(p.shape) == 3 else 4)
        maps = t(p.maps.astype(np.complex64))
        ctx.set_operator(maps, coords=t(p.coords.astype(np.float32)),
                         dcf=t(p.dcf.astype(np.float32)))
        m = maps[..., :C].contiguous()
        x = t(p.x_true.astype(np.complex64))
        outs = []
        for cfg in range(SPREAD_NCFG):
            ctx.set_spread_cfg(cfg)
            outs.append(ctx.normal_apply(m, x))
        for cfg in range(1, SPREAD_NCFG):
            assert torch.equal(outs[0], outs[cfg]), (name, cfg)
        best, ms = ctx.autotune_spread(m, reps=2)
        assert 0 <= best < SPREAD_NCFG and all(v > 0 for v in ms)
        assert ms[best] == min(ms)
        assert torch.equal(ctx.normal_apply(m, x), outs[0])
        ctx.close()
