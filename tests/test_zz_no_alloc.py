"""Allocation-free coil mixing (cs_coil_mix_noalloc) against the allocating
entry point cs_coil_mix: same kernel and fragments, so the outputs must be
bit-identical.  Two calls in a row, the second on smaller sizes, so that the
shared static scratch holds the first call's fragments when the second runs;
sizes beyond the scratch maximum are rejected before any device work."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import case, dev, t

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(shape, C):
    from paper_2305_06482_amd import Context
    return Context(shape, C, "cart", wav_levels=2)


def _rand_c(shape, seed):
    g = np.random.default_rng(seed)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / np.sqrt(2)


def _both(ctx, inp, M):
    ref = ctx.coil_mix(inp, M)
    Md = torch.from_numpy(np.ascontiguousarray(M)).to(torch.complex128).to(dev())
    out = torch.full(ref.shape, float("nan"), dtype=torch.complex64, device=dev())
    ctx.coil_mix_noalloc(inp, Md, out)
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_matches_coil_mix_two_calls():
    dev()
    shape = (40, 52)  # 2080 rows: 130 tiles of 16, a ragged last work-group
    ctx = _ctx(shape, 8)
    try:
        # first call: the largest size the scratch holds (64 -> 64 coils),
        # a general complex matrix (all three bf16 split terms non-zero)
        case("noalloc coil mix 64 -> 64, general M")
        inp = t(_rand_c(shape + (64,), 1))
        M = _rand_c((64, 64), 2)
        ref, out = _both(ctx, inp, M)
        assert torch.equal(ref, out)
        # second call, smaller: 26 -> 6 coils with +-1 / sqrt(6) entries (the
        # Rademacher block; the allocating entry point takes the one-term
        # path only when every entry is exact in bf16, here they are not) and
        # then +-1 entries (exact: one term there, three here)
        case("noalloc coil mix 26 -> 6, Rademacher / sqrt(S)")
        inp2 = t(_rand_c(shape + (26,), 3))
        R = np.where(np.random.default_rng(4).random((6, 26)) < 0.5, -1.0, 1.0)
        ref, out = _both(ctx, inp2, R / np.sqrt(6))
        assert torch.equal(ref, out)
        case("noalloc coil mix 26 -> 6, +-1 entries")
        ref, out = _both(ctx, inp2, R.astype(complex))
        assert torch.equal(ref, out)
        # the result is the mixing product itself (FP32 accuracy)
        want = np.einsum("...c,jc->...j", inp2.cpu().numpy().astype(np.complex128), R)
        got = out.cpu().numpy()
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-6
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    dev()
    shape = (16, 16)
    ctx = _ctx(shape, 4)
    try:
        lib = ctx.lib
        inp = t(_rand_c(shape + (65,), 5))
        M = torch.zeros((4, 65), dtype=torch.complex128, device=dev())
        out = torch.zeros(shape + (4,), dtype=torch.complex64, device=dev())
        rc = lib.cs_coil_mix_noalloc(ctx._ctx, ctypes.c_void_p(inp.data_ptr()), 65,
                                     ctypes.c_void_p(M.data_ptr()), 4,
                                     ctypes.c_void_p(out.data_ptr()))
        assert rc == -1
        assert b"[1, 64]" in lib.cs_last_error(ctx._ctx)
        rc = lib.cs_coil_mix_noalloc(ctx._ctx, ctypes.c_void_p(inp.data_ptr()), 4,
                                     ctypes.c_void_p(M.data_ptr()), 65,
                                     ctypes.c_void_p(out.data_ptr()))
        assert rc == -1
        torch.cuda.synchronize()
        assert bool((out == 0).all())  # nothing was written
    finally:
        ctx.close()
