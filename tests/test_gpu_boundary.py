"""The boundary calls that change where data comes from, against the FP64
oracle: a context built on a caller-owned workspace (cs_create_ws) gives the
same operator as one that allocates its own buffers; an injected PCA basis
and random block (cs_set_basis, cs_set_sketch; Sec. 2.3.2-2.3.3, Eqs. 11-13)
give the oracle's sketched maps for that basis and block; and the optional
reconstruction buffers reserved up front (cs_reserve_recon) leave the
reconstruction unchanged."""
import numpy as np
import pytest

import synth
from oracle import cartesian as cart
from oracle import nufft
from oracle import sketch as sk
from tests.gpu_helpers import case, dev, h, rel, rng_c, t

pytestmark = pytest.mark.gpu


def test_workspace_context_matches_allocating_context():
    dev()
    import torch
    from paper_2305_06482_amd import Context
    case("cs_create_ws 3D cones 16x24x24 C=5")
    shape = (16, 24, 24)
    coords = synth.cones_traj(shape, 120, 32, seed=3)
    dcf = synth.cones_dcf(coords, shape)
    maps = synth.coil_maps(shape, 5, 2)
    outs = []
    for ws in (False, True):
        ctx = Context(shape, 5, "noncart", nsamp=coords.shape[0], wav_levels=2, workspace=ws)
        assert (ctx.workspace is not None) == ws
        ctx.set_operator(t(maps), coords=t(coords.astype(np.float32)),
                         dcf=t(dcf.astype(np.float32)))
        x = synth.phantom(shape, 1)
        outs.append(h(ctx.normal_apply(t(maps), t(x))))
        ctx.close()
    assert np.array_equal(outs[0], outs[1])
    plan = nufft.Plan(shape, coords.astype(np.float32).astype(np.float64),
                      dcf.astype(np.float32).astype(np.float64))
    assert rel(outs[1], plan.normal(synth.phantom(shape, 1), maps)) < 1e-4
    torch.cuda.synchronize()


def test_injected_basis_and_block_give_the_oracle_sketch():
    dev()
    from paper_2305_06482_amd import Context
    case("cs_set_basis + cs_set_sketch 64x48 C=8 V=3 S=2")
    shape, C, V, S = (64, 48), 8, 3, 2
    maps = synth.coil_maps(shape, C, 5)
    mask = synth.mask_1d_vd(shape[0], shape[1], 6, n_center=8, accel=3)
    ctx = Context(shape, C, "cart", wav_levels=3)
    ctx.set_operator(t(maps), mask=t(mask, __import__("torch").uint8))
    # a basis that is not the data's PCA basis: a random unitary matrix
    g = np.random.default_rng(7)
    U, _ = np.linalg.qr(g.standard_normal((C, C)) + 1j * g.standard_normal((C, C)))
    R = g.choice([-1.0, 1.0], size=(S, C - V)) / np.sqrt(S)
    R[0, 1] = 0.75  # any real block, not only signs
    ctx.set_basis(U, np.arange(C, 0, -1, dtype=float))
    ctx.set_sketch(V, S, R)
    y = t(rng_c(shape + (C,), 8))  # data: ignored, the basis is cached
    sm, lam, Ug, signs = ctx.sketch_build(y, V, S, seed=3, t=4)
    want = sk.sketched_maps(sk.virtual_maps(maps, U), sk.sketch_matrix(V, S, C, R * np.sqrt(S)))
    assert rel(h(sm), want) < 1e-5
    assert np.allclose(Ug, U) and np.allclose(lam, np.arange(C, 0, -1))
    # the normal operator on the injected sketch
    z = synth.phantom(shape, 9)
    n = ctx.normal_apply(sm, t(z))
    assert rel(h(n), cart.normal(z, want, mask)) < 1e-4
    # back to the seeded draw: the oracle's Rademacher block of t = 4
    ctx.set_sketch(V, S, None)
    sm2, _, _, signs2 = ctx.sketch_build(y, V, S, seed=3, t=4)
    want2, ent = sk.sketch_for_iteration(sk.virtual_maps(maps, U), V, S, 3, 4)
    assert np.array_equal(signs2, ent.astype(np.int8))
    assert rel(h(sm2), want2) < 1e-5
    ctx.close()


def test_reserved_recon_buffers_leave_the_result_unchanged():
    dev()
    from paper_2305_06482_amd import Context
    case("cs_reserve_recon 64x64 C=8 C0=6 init")
    import torch
    shape, C = (64, 64), 8
    x = synth.phantom(shape, 11)
    maps = synth.coil_maps(shape, C, 12)
    mask = synth.mask_1d_vd(64, 64, 13, n_center=12, accel=4)
    y = cart.forward(x, maps, mask)
    for opts in ({"C0": 6}, {"init_iters": 2}):
        res = []
        for reserve in (False, True):
            ctx = Context(shape, C, "cart", wav_levels=4)
            ctx.set_operator(t(maps), mask=t(mask, torch.uint8))
            if reserve:
                ctx.reserve_recon(C0=6, init_coils=4)
            r = ctx.recon_run(t(y), mode="sketch", lam=1e-3, T=2, K=3, V=2, S=2, seed=5,
                              step=0.5, **opts)
            res.append(h(r.x))
            ctx.close()
        assert np.array_equal(res[0], res[1]), opts


def test_operator_setup_rejects_bad_trajectories():
    """The trajectory is checked on the GPU while it is binned: a coordinate
    outside [-n/2, n/2) or a negative density weight fails cs_set_operator
    with CS_EINVAL and its message, and a good trajectory set afterwards on
    the same context works."""
    dev()
    from paper_2305_06482_amd import Context
    from paper_2305_06482_amd.binding import CSError
    case("set_operator on bad trajectories (16x24x24, C=3)")
    shape = (16, 24, 24)
    coords = synth.cones_traj(shape, 40, 16, seed=8).astype(np.float32)
    dcf = synth.cones_dcf(coords, shape).astype(np.float32)
    maps = synth.coil_maps(shape, 3, 9)
    ctx = Context(shape, 3, "noncart", nsamp=coords.shape[0], wav_levels=2)
    bad = coords.copy()
    bad[17, 1] = 12.0  # y frequency n_y / 2: outside [-12, 12)
    with pytest.raises(CSError, match="coordinate outside"):
        ctx.set_operator(t(maps), coords=t(bad), dcf=t(dcf))
    badw = dcf.copy()
    badw[5] = -1.0
    with pytest.raises(CSError, match="density compensation"):
        ctx.set_operator(t(maps), coords=t(coords), dcf=t(badw))
    with pytest.raises(CSError, match="cs_set_operator has not been called"):
        ctx.normal_apply(t(maps), t(synth.phantom(shape, 2)))
    ctx.set_operator(t(maps), coords=t(coords), dcf=t(dcf))
    plan = nufft.Plan(shape, coords.astype(np.float64), dcf.astype(np.float64))
    x = synth.phantom(shape, 2)
    assert rel(h(ctx.normal_apply(t(maps), t(x))), plan.normal(x, maps)) < 1e-4
    ctx.close()
