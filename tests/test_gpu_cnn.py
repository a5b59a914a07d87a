"""The learned warm start on the GPU: BF16-MFMA forward and gradients against
the FP64 reference network, training, the solver-pair collector, the
fallback under a garbage network, and what a trained network gains."""
import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
from tests.gpu_helpers import case, dev, h, t

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def net():
    dev()
    import torch
    from paper_2305_06482_amd import CNN
    n = CNN(seed=11)
    yield torch, n
    n.close()


def test_forward_matches_fp64_reference(net):
    torch, n = net
    case("CNN forward vs FP64 reference, 6x10x20 (ragged x tile)")
    rng = np.random.default_rng(0)
    p = n.get_params().astype(np.float64)
    assert p.size == ocnn.n_params()
    x = rng.standard_normal((6, 10, 20, 4)).astype(np.float32)
    got = h(n.forward(t(x)))
    ref = ocnn.forward(p, x.astype(np.float64))
    e = _rel(got, ref)
    assert e < 2e-2, e  # BF16 operands (8-bit mantissa), FP32 accumulation


def test_gradients_match_fp64_reference(net):
    torch, n = net
    case("CNN loss and gradients vs FP64 reference")
    rng = np.random.default_rng(1)
    p = (rng.standard_normal(ocnn.n_params()) * 0.05).astype(np.float32)
    n.set_params(p)
    x = rng.standard_normal((5, 8, 16, 4)).astype(np.float32)
    tg = rng.standard_normal((5, 8, 16, 2)).astype(np.float32)
    loss = n.loss_grad(t(x), t(tg))
    g = n.get_grads()
    L, gref = ocnn.loss_grad(p.astype(np.float64), x.astype(np.float64), tg.astype(np.float64))
    assert abs(loss - L) < 1e-2 * L, (loss, L)
    e = _rel(g, gref)
    assert e < 5e-2, e
    # per layer, the weight block and the bias block
    off = 0
    for cin, cout in zip(ocnn.WIDTHS[:-1], ocnn.WIDTHS[1:]):
        nw = 27 * cin * cout
        ew = _rel(g[off:off + nw], gref[off:off + nw])
        eb = _rel(g[off + nw:off + nw + cout], gref[off + nw:off + nw + cout])
        # BF16 operands (relative rounding 2^-9 each) through up to three
        # backward layers, plus ReLU masks that flip where a pre-activation
        # is within rounding of zero: a few percent per block
        assert ew < 1e-1 and eb < 1e-1, (cin, cout, ew, eb)
        off += nw + cout


def test_training_fits_a_target_network(net):
    torch, n = net
    case("CNN training fits a reachable target")
    rng = np.random.default_rng(2)
    teacher = rng.standard_normal(ocnn.n_params()) * 0.06
    xs = [rng.standard_normal((8, 16, 16, 4)) for _ in range(4)]
    ys = [ocnn.forward(teacher, x) for x in xs]
    from paper_2305_06482_amd import CNN
    s = CNN(seed=5)
    losses = []
    for step in range(150):
        i = step % 4
        losses.append(s.train_step(t(xs[i].astype(np.float32)), t(ys[i].astype(np.float32)),
                                   2e-3))
    s.close()
    first, last = np.mean(losses[:8]), np.mean(losses[-8:])
    assert np.isfinite(last) and last < 0.5 * first, (first, last)


def _radial(n_img=64, seed=5300):
    import torch
    from paper_2305_06482_amd import Context
    p = synth.make_radial(n_img, 48, 8, 2, 2, seed_base=seed)
    ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0], wav_levels=4)
    maps = t(p.maps.astype(np.complex64))
    dcf = t(p.dcf.astype(np.float32))
    ctx.set_operator(maps, coords=t(p.coords.astype(np.float32)), dcf=dcf)
    y = ctx.sense_apply(maps, t(p.x_true.astype(np.complex64)))
    y += t(p.noise.astype(np.complex64)) * dcf.sqrt()[:, None].to(torch.complex64)
    return p, ctx, y


def test_collector_follows_the_solver():
    dev()
    import torch
    case("solver-pair collector vs recon_run")
    p, ctx, y = _radial()
    inp, tgt, xc = ctx.collect(y, 3, 4, p.V, p.S, p.seed, p.lam)
    r = ctx.recon_run(y, mode="sketch", lam=p.lam, T=3, K=4, V=p.V, S=p.S, seed=p.seed)
    assert torch.equal(xc, r.x)
    assert inp.shape == (3, 1, 64, 64, 4) and tgt.shape == (3, 1, 64, 64, 2)
    assert torch.isfinite(inp).all() and torch.isfinite(tgt).all()
    # target 0 is x^1 / s_o (x^0 = 0) and input 0 carries x^0 = 0
    assert float(inp[0, ..., :2].abs().max()) == 0.0
    r1 = ctx.recon_run(y, mode="sketch", lam=p.lam, T=1, K=4, V=p.V, S=p.S, seed=p.seed)
    x1 = torch.view_as_real(r1.x)[None]
    ratio = (tgt[0][x1 != 0] / x1[x1 != 0])
    assert float(ratio.std() / ratio.mean().abs()) < 1e-5  # one common scale 1 / s_o
    ctx.close()


def test_garbage_network_falls_back_to_the_plain_method():
    dev()
    import torch
    from paper_2305_06482_amd import CNN
    case("learned mode with a garbage network: every warm start rejected")
    p, ctx, y = _radial(seed=5310)
    bad = CNN(seed=3)
    bad.set_params(np.full(bad.num_params, 50.0, dtype=np.float32))
    T, K = 4, 4
    r0 = ctx.recon_run(y, mode="sketch", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed)
    r1 = ctx.recon_run(y, mode="learned", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed,
                       cnn=bad)
    assert r1.n_warm_rejected == T and r1.n_warm_accepted == 0
    assert torch.equal(r0.x, r1.x)
    # the objective monitor in learned mode only reads: with a tolerance no
    # outer step reaches, nothing falls back and x is unchanged
    r2 = ctx.recon_run(y, mode="learned", lam=p.lam, T=T, K=K, V=p.V, S=p.S, seed=p.seed,
                       cnn=bad, monitor=True, mon_tol=0.5)
    assert r2.n_fallbacks == 0 and r2.n_warm_rejected == T
    assert len(r2.objective) == T and np.all(np.isfinite(r2.objective))
    assert r2.objective[-1] < r2.objective0
    assert torch.equal(r0.x, r2.x)
    bad.close()
    ctx.close()


def test_trained_network_gain_on_held_out_cones():
    """Trains on pairs from 6 small cones problems and compares plain and
    learned Algorithm 1 on 2 held-out ones (distance to the full-coil
    minimizer after T outer iterations).  The fallback guarantees the
    learned run is never driven off by the network; the measured gain is
    printed."""
    dev()
    import torch
    from paper_2305_06482_amd import CNN, Context, learned
    case("learned warm start: train on 6 cones problems, test on 2 held out")
    T, K = 6, 5

    def problem(seed):
        p = synth.make_cones(shape=(32, 32, 32), n_readouts=600, n_samples=96, n_coils=16,
                             V=4, S=4, seed_base=seed, lam=5e-4)
        ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0], wav_levels=3)
        maps = t(p.maps.astype(np.complex64))
        dcf = t(p.dcf.astype(np.float32))
        ctx.set_operator(maps, coords=t(p.coords.astype(np.float32)), dcf=dcf)
        y = ctx.sense_apply(maps, t(p.x_true.astype(np.complex64)))
        y += t(p.noise.astype(np.complex64)) * dcf.sqrt()[:, None].to(torch.complex64)
        return p, ctx, y

    train_set = [problem(9000 + 10 * i) for i in range(6)]
    ins, tgts = learned.collect_pairs(
        [(c, y, p.V, p.S, p.seed, p.lam) for p, c, y in train_set], T, K)
    net = CNN(seed=21)
    losses = learned.train(net, ins, tgts, 600, patch=(32, 32, 32), lr=1e-3)
    assert np.mean(losses[-20:]) < np.mean(losses[:20])
    for _, c, _ in train_set:
        c.close()
    gains = []
    for seed in (9500, 9510):
        p, ctx, y = problem(seed)
        x_inf = ctx.recon_run(y, mode="full", lam=p.lam, T=3000, step=0.0).x
        ev = learned.evaluate(ctx, y, x_inf, net, T, K, p.V, p.S, p.seed, p.lam)
        d0, d1 = ev["sketch"]["dist"][-1], ev["learned"]["dist"][-1]
        gains.append(d0 / d1)
        print(f"held-out {seed}: plain d={d0:.4g}, learned d={d1:.4g} "
              f"(accepted {ev['learned']['accepted']}/{T})", flush=True)
        assert d1 <= 1.05 * d0, (d0, d1)
        ctx.close()
    print(f"distance ratio plain/learned after {T} outer iterations: {gains}", flush=True)
    net.close()
