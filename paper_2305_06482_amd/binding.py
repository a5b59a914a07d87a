"""Thin ctypes binding over ``libcoilsketch.so`` (argument marshalling only).

Every call forwards device pointers of caller-owned PyTorch tensors and the
context's HIP stream to the C ABI declared in ``include/coilsketch.h``; all
arithmetic runs in the library's HIP kernels.  There is no fallback: if the
library is missing or a call fails, an exception is raised.

Layouts (see the header): images are complex64 row-major ``(nz, ny, nx)`` or
``(ny, nx)``; coil stacks are pixel-major with the coil index fastest
(``maps[..., c]``, data ``[N, C]``); coordinates are float32 ``[N, ndim]`` in
cycles/FOV with column 0 the x frequency.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# COILSKETCH_LIB in the environment names another build of the library
LIB_PATH = os.environ.get("COILSKETCH_LIB") or os.path.join(_HERE, "libcoilsketch.so")

CS_CART = 0
CS_NONCART = 1
CS_RECON_FULL = 0
CS_RECON_SKETCH = 1
CS_RECON_SKETCH_LEARNED = 2
CS_REG_L1WAV, CS_REG_L2, CS_REG_TV = 0, 1, 2
CS_SKETCH_RADEMACHER, CS_SKETCH_GAUSSIAN = 0, 1

EXPORTED = [
    "cs_create", "cs_create_ws", "cs_workspace_size", "cs_destroy", "cs_last_error", "cs_set_operator", "sense_apply",
    "sense_adjoint", "normal_apply", "sketch_build", "recon_run", "cs_prox_l1wav",
    "cs_dwt", "cs_idwt", "cs_coil_mix", "cs_coil_mix_noalloc", "cs_dot", "cs_power_iteration", "cs_grid_shape",
    "cs_profile_enable", "cs_profile_read", "cs_batch_create", "cs_batch_destroy",
    "cs_batch_last_error", "cs_batch_recon", "cs_set_spread_cfg", "cs_autotune_spread",
    "cs_set_interp_cfg", "cs_set_sketch_dist", "cs_set_basis", "cs_set_sketch",
    "cs_reserve_recon",
    "cs_cnn_create", "cs_cnn_destroy", "cs_cnn_last_error", "cs_cnn_num_params",
    "cs_cnn_get_params", "cs_cnn_set_params", "cs_cnn_forward", "cs_cnn_loss_grad",
    "cs_cnn_train_step", "cs_cnn_collect",
]
SPREAD_NCFG = 13
INTERP_NCFG = 5
NKERNELS = 12
KERNEL_KINDS = ["fft_pass", "interp", "spread", "gather", "wavelet", "soft", "vec", "reduce",
                "covariance", "eigensolver", "coil_mix", "spread_merge"]


class CSError(RuntimeError):
    pass


class Geom(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("ncoil", ctypes.c_int),
        ("kind", ctypes.c_int),
        ("nsamp", ctypes.c_longlong),
        ("sigma", ctypes.c_float),
        ("kwidth", ctypes.c_int),
        ("beta", ctypes.c_float),
        ("wav_levels", ctypes.c_int),
    ]


class ReconParams(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int),
        ("lam", ctypes.c_float),
        ("T", ctypes.c_int),
        ("K", ctypes.c_int),
        ("V", ctypes.c_int),
        ("S", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("t0", ctypes.c_int),
        ("step", ctypes.c_double),
        ("n_pow", ctypes.c_int),
        ("reuse_b", ctypes.c_int),
        ("x_ref", ctypes.c_void_p),
        ("cnn", ctypes.c_void_p),
        ("reg", ctypes.c_int),
        ("n_cg", ctypes.c_int),
        ("init_iters", ctypes.c_int),
        ("C0", ctypes.c_int),
        ("monitor", ctypes.c_int),
        ("mon_tol", ctypes.c_double),
    ]


class ReconStats(ctypes.Structure):
    _fields_ = [
        ("dist", ctypes.POINTER(ctypes.c_double)),
        ("time_ms", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double),
        ("n_full_applies", ctypes.c_longlong),
        ("n_sketch_applies", ctypes.c_longlong),
        ("n_prox", ctypes.c_longlong),
        ("total_ms", ctypes.c_double),
        ("ms_full_normal", ctypes.c_double),
        ("ms_sketch_normal", ctypes.c_double),
        ("ms_prox", ctypes.c_double),
        ("ms_sketch", ctypes.c_double),
        ("prep_ms", ctypes.c_double),
        ("n_warm_accepted", ctypes.c_longlong),
        ("n_warm_rejected", ctypes.c_longlong),
        ("ms_warm", ctypes.c_double),
        ("objective", ctypes.POINTER(ctypes.c_double)),
        ("objective0", ctypes.c_double),
        ("n_fallbacks", ctypes.c_longlong),
        ("ms_monitor", ctypes.c_double),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double),
        ("n_full_applies", ctypes.c_longlong),
        ("n_sketch_applies", ctypes.c_longlong),
        ("wall_prep_ms", ctypes.c_double),
        ("wall_loop_ms", ctypes.c_double),
        ("graph_nodes", ctypes.c_longlong),
        ("graph_replays", ctypes.c_longlong),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CSError(f"{LIB_PATH} not found: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cf, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
    lib.cs_create.argtypes = [ctypes.POINTER(Geom), vp, ctypes.POINTER(vp)]
    lib.cs_create_ws.argtypes = [ctypes.POINTER(Geom), vp, ctypes.c_size_t, vp,
                                 ctypes.POINTER(vp)]
    lib.cs_workspace_size.argtypes = [ctypes.POINTER(Geom), ctypes.POINTER(ctypes.c_size_t)]
    lib.cs_set_basis.argtypes = [vp, vp, vp]
    lib.cs_set_sketch.argtypes = [vp, ci, ci, vp]
    lib.cs_reserve_recon.argtypes = [vp, ci, ci]
    lib.cs_destroy.argtypes = [vp]
    lib.cs_destroy.restype = None
    lib.cs_last_error.argtypes = [vp]
    lib.cs_last_error.restype = ctypes.c_char_p
    lib.cs_set_operator.argtypes = [vp, vp, vp, vp, vp]
    for name in ("sense_apply", "sense_adjoint", "normal_apply"):
        getattr(lib, name).argtypes = [vp, vp, ci, vp, vp]
    lib.sketch_build.argtypes = [vp, vp, ci, ci, ctypes.c_uint64, ci, ci, vp, vp, vp, vp]
    lib.recon_run.argtypes = [vp, vp, ctypes.POINTER(ReconParams), vp,
                              ctypes.POINTER(ReconStats)]
    lib.cs_prox_l1wav.argtypes = [vp, vp, cf, vp]
    lib.cs_dwt.argtypes = [vp, vp, vp]
    lib.cs_idwt.argtypes = [vp, vp, vp]
    lib.cs_coil_mix.argtypes = [vp, vp, ci, vp, ci, vp]
    lib.cs_coil_mix_noalloc.argtypes = [vp, vp, ci, vp, ci, vp]
    lib.cs_dot.argtypes = [vp, vp, vp, vp]
    lib.cs_power_iteration.argtypes = [vp, vp, ci, ci, vp]
    lib.cs_grid_shape.argtypes = [vp, vp]
    lib.cs_profile_enable.argtypes = [vp, ci]
    lib.cs_profile_read.argtypes = [vp, vp, vp]
    lib.cs_batch_create.argtypes = [vp, ci, vp, ctypes.POINTER(vp)]
    lib.cs_batch_destroy.argtypes = [vp]
    lib.cs_batch_destroy.restype = None
    lib.cs_batch_last_error.argtypes = [vp]
    lib.cs_batch_last_error.restype = ctypes.c_char_p
    lib.cs_batch_recon.argtypes = [vp, vp, ctypes.POINTER(ReconParams), vp, ci,
                                   ctypes.POINTER(BatchStats)]
    lib.cs_set_spread_cfg.argtypes = [vp, ci]
    lib.cs_set_interp_cfg.argtypes = [vp, ci]
    lib.cs_set_sketch_dist.argtypes = [vp, ci]
    lib.cs_autotune_spread.argtypes = [vp, vp, ci, ci, ctypes.POINTER(ci), vp]
    lib.cs_cnn_create.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
    lib.cs_cnn_destroy.argtypes = [vp]
    lib.cs_cnn_destroy.restype = None
    lib.cs_cnn_last_error.argtypes = [vp]
    lib.cs_cnn_last_error.restype = ctypes.c_char_p
    lib.cs_cnn_num_params.argtypes = [vp]
    lib.cs_cnn_get_params.argtypes = [vp, vp, vp]
    lib.cs_cnn_set_params.argtypes = [vp, vp]
    lib.cs_cnn_forward.argtypes = [vp, vp, ci, ci, ci, vp]
    lib.cs_cnn_loss_grad.argtypes = [vp, vp, vp, ci, ci, ci, ctypes.POINTER(cd)]
    lib.cs_cnn_train_step.argtypes = [vp, vp, vp, ci, ci, ci, cf, ctypes.POINTER(cd)]
    lib.cs_cnn_collect.argtypes = [vp, vp, ctypes.POINTER(ReconParams), vp, vp, vp]
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("cs_destroy", "cs_last_error", "cs_batch_destroy",
                        "cs_batch_last_error", "cs_cnn_destroy", "cs_cnn_last_error",
                        "cs_cnn_num_params"):
            f.restype = ci
    lib.cs_cnn_num_params.restype = ctypes.c_longlong
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


@dataclass
class ReconResult:
    x: torch.Tensor
    alpha: float
    n_full_applies: int
    n_sketch_applies: int
    n_prox: int
    total_ms: float
    ms_full_normal: float = 0.0
    ms_sketch_normal: float = 0.0
    ms_prox: float = 0.0
    ms_sketch: float = 0.0
    prep_ms: float = 0.0
    n_warm_accepted: int = 0
    n_warm_rejected: int = 0
    ms_warm: float = 0.0
    time_ms: list = field(default_factory=list)
    dist: list = field(default_factory=list)
    objective0: float = 0.0
    objective: list = field(default_factory=list)
    n_fallbacks: int = 0
    ms_monitor: float = 0.0


def _geom(shape, ncoil, kind="cart", nsamp=0, sigma=1.25, kwidth=4, beta=0.0, wav_levels=4):
    g = Geom()
    g.ndim = len(shape)
    for i, s in enumerate(shape):
        g.n[i] = int(s)
    g.ncoil = int(ncoil)
    g.kind = CS_CART if kind == "cart" else CS_NONCART
    g.nsamp = int(nsamp)
    g.sigma = float(sigma)
    g.kwidth = int(kwidth)
    g.beta = float(beta)
    g.wav_levels = int(wav_levels)
    return g


def workspace_size(shape, ncoil, kind="cart", nsamp=0, sigma=1.25, kwidth=4, beta=0.0,
                   wav_levels=4):
    """cs_workspace_size for a geometry (no device work)."""
    lib = load()
    g = _geom(shape, ncoil, kind, nsamp, sigma, kwidth, beta, wav_levels)
    nb = ctypes.c_size_t()
    rc = lib.cs_workspace_size(ctypes.byref(g), ctypes.byref(nb))
    if rc != 0:
        raise CSError(f"cs_workspace_size failed ({rc}): {lib.cs_last_error(None).decode()}")
    return int(nb.value)


class Context:
    """One operator geometry bound to the current HIP stream."""

    def __init__(self, shape, ncoil, kind="cart", nsamp=0, sigma=1.25, kwidth=4,
                 beta=0.0, wav_levels=4, device=None, workspace=False):
        """workspace=True: the work buffers come from a torch byte tensor of
        cs_workspace_size() bytes held by this object (cs_create_ws)."""
        self.lib = load()
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.C = int(ncoil)
        self.kind = CS_CART if kind == "cart" else CS_NONCART
        self.N = int(nsamp) if self.kind == CS_NONCART else int(torch.tensor(self.shape).prod())
        self.device = torch.device(device or "cuda")
        self.stream = torch.cuda.current_stream(self.device)
        g = Geom()
        g.ndim = self.ndim
        for i, s in enumerate(self.shape):
            g.n[i] = s
        g.ncoil = self.C
        g.kind = self.kind
        g.nsamp = int(nsamp)
        g.sigma = float(sigma)
        g.kwidth = int(kwidth)
        g.beta = float(beta)
        g.wav_levels = int(wav_levels)
        self._ctx = ctypes.c_void_p()
        self.workspace = None
        if workspace:
            nb = workspace_size(self.shape, ncoil, kind, nsamp, sigma, kwidth, beta, wav_levels)
            # torch's caching allocator hands out 512-byte aligned blocks
            self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
            rc = self.lib.cs_create_ws(ctypes.byref(g), _ptr(self.workspace), nb,
                                       ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(self._ctx))
        else:
            rc = self.lib.cs_create(ctypes.byref(g), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(self._ctx))
        if rc != 0:
            raise CSError(f"cs_create failed ({rc}): {self.lib.cs_last_error(None).decode()}")
        self._keep = {}

    # -- helpers -----------------------------------------------------------
    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.cs_last_error(self._ctx).decode()
            raise CSError(f"{what} failed ({rc}): {msg}")

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.cs_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _img(self, t, name):
        _need(t, torch.complex64, self.shape, name)

    def _maps(self, maps, name="maps"):
        _need(maps, torch.complex64, None, name)
        if tuple(maps.shape[:-1]) != self.shape:
            raise ValueError(f"{name} must have shape image + (ncoil,)")
        return int(maps.shape[-1])

    def _data(self, y, ncoil, name="y"):
        _need(y, torch.complex64, None, name)
        if self.kind == CS_CART:
            ok = tuple(y.shape) == self.shape + (ncoil,)
        else:
            ok = tuple(y.shape) == (self.N, ncoil)
        if not ok:
            raise ValueError(f"{name} has shape {tuple(y.shape)}")

    def empty_image(self):
        return torch.empty(self.shape, dtype=torch.complex64, device=self.device)

    def empty_data(self, ncoil):
        if self.kind == CS_CART:
            return torch.empty(self.shape + (ncoil,), dtype=torch.complex64, device=self.device)
        return torch.empty((self.N, ncoil), dtype=torch.complex64, device=self.device)

    # -- C ABI ----------------------------------------------------------------
    def set_operator(self, maps, mask=None, coords=None, dcf=None):
        self._maps(maps)
        if self.kind == CS_CART:
            _need(mask, torch.uint8, self.shape, "mask")
        else:
            _need(coords, torch.float32, (self.N, self.ndim), "coords")
            if dcf is not None:
                _need(dcf, torch.float32, (self.N,), "dcf")
        self._keep["maps"] = maps
        self._check(self.lib.cs_set_operator(self._ctx, _ptr(maps), _ptr(mask), _ptr(coords),
                                             _ptr(dcf)), "cs_set_operator")

    def sense_apply(self, maps, x, y=None):
        nc = self._maps(maps)
        self._img(x, "x")
        y = self.empty_data(nc) if y is None else y
        self._data(y, nc)
        self._check(self.lib.sense_apply(self._ctx, _ptr(maps), nc, _ptr(x), _ptr(y)),
                    "sense_apply")
        return y

    def sense_adjoint(self, maps, y, x=None):
        nc = self._maps(maps)
        self._data(y, nc)
        x = self.empty_image() if x is None else x
        self._img(x, "x")
        self._check(self.lib.sense_adjoint(self._ctx, _ptr(maps), nc, _ptr(y), _ptr(x)),
                    "sense_adjoint")
        return x

    def normal_apply(self, maps, x, out=None):
        nc = self._maps(maps)
        self._img(x, "x")
        out = self.empty_image() if out is None else out
        self._img(out, "out")
        self._check(self.lib.normal_apply(self._ctx, _ptr(maps), nc, _ptr(x), _ptr(out)),
                    "normal_apply")
        return out

    def sketch_build(self, y, V, S, seed, t, refresh=False, smaps=None, host_outputs=True):
        self._data(y, self.C)
        Ch = V + S
        smaps = (torch.empty(self.shape + (Ch,), dtype=torch.complex64, device=self.device)
                 if smaps is None else smaps)
        _need(smaps, torch.complex64, self.shape + (Ch,), "smaps")
        eig = U = signs = None
        if host_outputs:
            eig = (ctypes.c_double * self.C)()
            U = (ctypes.c_double * (2 * self.C * self.C))()
            signs = (ctypes.c_int8 * max(1, S * (self.C - V)))()
        rc = self.lib.sketch_build(self._ctx, _ptr(y), int(V), int(S), ctypes.c_uint64(seed),
                                   int(t), int(bool(refresh)), _ptr(smaps),
                                   eig and ctypes.cast(eig, ctypes.c_void_p),
                                   U and ctypes.cast(U, ctypes.c_void_p),
                                   signs and ctypes.cast(signs, ctypes.c_void_p))
        self._check(rc, "sketch_build")
        if not host_outputs:
            return smaps, None, None, None
        import numpy as np
        lam = np.array(eig[:], dtype=np.float64)
        Uc = np.array(U[:], dtype=np.float64).reshape(self.C, self.C, 2)
        Uc = Uc[..., 0] + 1j * Uc[..., 1]
        sg = np.array(signs[:S * (self.C - V)], dtype=np.int8).reshape(S, self.C - V)
        return smaps, lam, Uc, sg

    def recon_run(self, y, mode="sketch", lam=1e-3, T=10, K=5, V=2, S=2, seed=0, t0=1,
                  step=0.0, n_pow=30, reuse_b=False, x=None, x_ref=None, cnn=None,
                  reg="l1wav", n_cg=5, init_iters=0, C0=0, monitor=False, mon_tol=1e-4):
        """Algorithm 1 (mode "sketch", "learned") or the plain solver ("full")
        with regularizer reg: "l1wav" (FISTA), "l2" (conjugate gradients) or
        "tv" (PDHG with n_cg CG iterations per data-consistency step).
        init_iters > 0 runs the classical-sketch initialisation first; 0 < C0 < C
        compresses to the first C0 virtual coils (Alg. 1's compression step).
        monitor=True evaluates the FP64 objective of every outer iterate and
        replaces one that rose by more than mon_tol (relative) or is not
        finite with a full-coil proximal-gradient step (l1wav Algorithm 1)."""
        self._data(y, self.C)
        if x is None:
            x = torch.zeros(self.shape, dtype=torch.complex64, device=self.device)
        self._img(x, "x")
        if x_ref is not None:
            self._img(x_ref, "x_ref")
        p = ReconParams()
        p.mode = {"sketch": CS_RECON_SKETCH, "full": CS_RECON_FULL,
                  "learned": CS_RECON_SKETCH_LEARNED}[mode]
        p.cnn = None if cnn is None else cnn._n.value
        p.reg = {"l1wav": CS_REG_L1WAV, "l2": CS_REG_L2, "tv": CS_REG_TV}[reg]
        p.n_cg = int(n_cg)
        p.init_iters = int(init_iters)
        p.C0 = int(C0)
        p.monitor = int(bool(monitor))
        p.mon_tol = float(mon_tol)
        p.lam = float(lam)
        p.T, p.K, p.V, p.S = int(T), int(K), int(V), int(S)
        p.seed = int(seed)
        p.t0 = int(t0)
        p.step = float(step)
        p.n_pow = int(n_pow)
        p.reuse_b = int(bool(reuse_b))
        p.x_ref = None if x_ref is None else x_ref.data_ptr()
        n = max(1, int(T))
        dist = (ctypes.c_double * n)()
        tms = (ctypes.c_double * n)()
        obj = (ctypes.c_double * n)()
        st = ReconStats()
        st.dist = ctypes.cast(dist, ctypes.POINTER(ctypes.c_double))
        st.time_ms = ctypes.cast(tms, ctypes.POINTER(ctypes.c_double))
        st.objective = ctypes.cast(obj, ctypes.POINTER(ctypes.c_double))
        self._check(self.lib.recon_run(self._ctx, _ptr(y), ctypes.byref(p), _ptr(x),
                                       ctypes.byref(st)), "recon_run")
        return ReconResult(x=x, alpha=st.alpha, n_full_applies=st.n_full_applies,
                           n_sketch_applies=st.n_sketch_applies, n_prox=st.n_prox,
                           total_ms=st.total_ms, ms_full_normal=st.ms_full_normal,
                           ms_sketch_normal=st.ms_sketch_normal, ms_prox=st.ms_prox,
                           ms_sketch=st.ms_sketch, prep_ms=st.prep_ms,
                           n_warm_accepted=st.n_warm_accepted,
                           n_warm_rejected=st.n_warm_rejected, ms_warm=st.ms_warm,
                           time_ms=list(tms[:T]),
                           dist=list(dist[:T]) if x_ref is not None else [],
                           objective0=st.objective0,
                           objective=list(obj[:T]) if monitor else [],
                           n_fallbacks=st.n_fallbacks, ms_monitor=st.ms_monitor)

    def prox_l1wav(self, v, tau, out=None):
        self._img(v, "v")
        out = self.empty_image() if out is None else out
        self._check(self.lib.cs_prox_l1wav(self._ctx, _ptr(v), ctypes.c_float(tau), _ptr(out)),
                    "cs_prox_l1wav")
        return out

    def dwt(self, x, out=None):
        self._img(x, "x")
        out = self.empty_image() if out is None else out
        self._check(self.lib.cs_dwt(self._ctx, _ptr(x), _ptr(out)), "cs_dwt")
        return out

    def idwt(self, c, out=None):
        self._img(c, "coef")
        out = self.empty_image() if out is None else out
        self._check(self.lib.cs_idwt(self._ctx, _ptr(c), _ptr(out)), "cs_idwt")
        return out

    def coil_mix(self, inp, M, out=None):
        """out[..., j] = sum_c inp[..., c] M[j, c] (M: complex numpy [cout, cin])."""
        import numpy as np
        cin = self._maps(inp, "inp")
        M = np.ascontiguousarray(np.asarray(M, dtype=np.complex128))
        cout = M.shape[0]
        if M.shape != (cout, cin):
            raise ValueError("M must be [cout, cin]")
        Mr = np.ascontiguousarray(np.stack([M.real, M.imag], -1))
        out = (torch.empty(self.shape + (cout,), dtype=torch.complex64, device=self.device)
               if out is None else out)
        _need(out, torch.complex64, self.shape + (cout,), "out")
        self._check(self.lib.cs_coil_mix(self._ctx, _ptr(inp), cin,
                                         Mr.ctypes.data_as(ctypes.c_void_p), cout, _ptr(out)),
                    "cs_coil_mix")
        return out

    def set_basis(self, U, lam=None):
        """cs_set_basis: U complex [C, C] (column j = eigenvector j)."""
        import numpy as np
        U = np.asarray(U, dtype=np.complex128)
        if U.shape != (self.C, self.C):
            raise ValueError("U must be [C, C]")
        Ur = np.ascontiguousarray(np.stack([U.real, U.imag], -1))
        lr = None if lam is None else np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
        if lr is not None and lr.shape != (self.C,):
            raise ValueError("lam must be [C]")
        self._check(self.lib.cs_set_basis(
            self._ctx, Ur.ctypes.data_as(ctypes.c_void_p),
            None if lr is None else lr.ctypes.data_as(ctypes.c_void_p)), "cs_set_basis")

    def set_sketch(self, V, S, R=None):
        """cs_set_sketch: R real [S, C - V] used as given; None returns to the draw."""
        import numpy as np
        if R is None:
            self._check(self.lib.cs_set_sketch(self._ctx, int(V), int(S), None), "cs_set_sketch")
            return
        R = np.ascontiguousarray(np.asarray(R, dtype=np.float64))
        if R.shape != (S, self.C - V):
            raise ValueError("R must be [S, C - V]")
        self._check(self.lib.cs_set_sketch(self._ctx, int(V), int(S),
                                           R.ctypes.data_as(ctypes.c_void_p)), "cs_set_sketch")

    def reserve_recon(self, C0=0, init_coils=0):
        self._check(self.lib.cs_reserve_recon(self._ctx, int(C0), int(init_coils)),
                    "cs_reserve_recon")

    def coil_mix_noalloc(self, inp, M, out):
        """cs_coil_mix_noalloc: M a device complex128 tensor [cout, cin]; out
        (device complex64 image + (cout,)) is caller-allocated, as the call
        itself allocates nothing."""
        cin = self._maps(inp, "inp")
        _need(M, torch.complex128, None, "M")
        if M.dim() != 2 or int(M.shape[1]) != cin:
            raise ValueError("M must be [cout, cin]")
        cout = int(M.shape[0])
        _need(out, torch.complex64, None, "out")
        if tuple(out.shape) != self.shape + (cout,):
            raise ValueError("out must have shape image + (cout,)")
        self._check(self.lib.cs_coil_mix_noalloc(self._ctx, _ptr(inp), cin, _ptr(M),
                                                 cout, _ptr(out)), "cs_coil_mix_noalloc")
        return out

    def dot(self, a, b):
        self._img(a, "a")
        self._img(b, "b")
        out = (ctypes.c_double * 2)()
        self._check(self.lib.cs_dot(self._ctx, _ptr(a), _ptr(b), ctypes.cast(out, ctypes.c_void_p)),
                    "cs_dot")
        return complex(out[0], out[1])

    def power_iteration(self, maps, n_iter=30):
        nc = self._maps(maps)
        L = ctypes.c_double()
        self._check(self.lib.cs_power_iteration(self._ctx, _ptr(maps), nc, int(n_iter),
                                                ctypes.byref(L)), "cs_power_iteration")
        return L.value

    def grid_shape(self):
        m = (ctypes.c_int * 3)()
        self._check(self.lib.cs_grid_shape(self._ctx, ctypes.cast(m, ctypes.c_void_p)),
                    "cs_grid_shape")
        return tuple(m[:])

    def profile_enable(self, on=True):
        self._check(self.lib.cs_profile_enable(self._ctx, int(bool(on))), "cs_profile_enable")

    def profile_read(self):
        """{kernel kind: (total ms, launches)} since the last read."""
        ms = (ctypes.c_double * NKERNELS)()
        cnt = (ctypes.c_longlong * NKERNELS)()
        self._check(self.lib.cs_profile_read(self._ctx, ctypes.cast(ms, ctypes.c_void_p),
                                             ctypes.cast(cnt, ctypes.c_void_p)),
                    "cs_profile_read")
        return {KERNEL_KINDS[i]: (ms[i], cnt[i]) for i in range(NKERNELS)}

    def collect(self, y, T, K, V, S, seed, lam, t0=1, step=0.0, n_pow=30, x=None):
        """Training pairs from T outer iterations of Algorithm 1: returns
        (inputs [T, *shape, 4], targets [T, *shape, 2]) as float32 tensors
        (2D images get a unit z axis), and the final iterate."""
        self._data(y, self.C)
        if x is None:
            x = torch.zeros(self.shape, dtype=torch.complex64, device=self.device)
        self._img(x, "x")
        vol = self.shape if self.ndim == 3 else (1,) + self.shape
        inp = torch.empty((T,) + vol + (4,), dtype=torch.float32, device=self.device)
        tgt = torch.empty((T,) + vol + (2,), dtype=torch.float32, device=self.device)
        p = ReconParams()
        p.mode = CS_RECON_SKETCH
        p.lam = float(lam)
        p.T, p.K, p.V, p.S = int(T), int(K), int(V), int(S)
        p.seed = int(seed)
        p.t0 = int(t0)
        p.step = float(step)
        p.n_pow = int(n_pow)
        self._check(self.lib.cs_cnn_collect(self._ctx, _ptr(y), ctypes.byref(p), _ptr(x),
                                            _ptr(inp), _ptr(tgt)), "cs_cnn_collect")
        return inp, tgt, x

    def set_spread_cfg(self, cfg):
        """Select a spreading work-group shape (0 .. SPREAD_NCFG - 1)."""
        self._check(self.lib.cs_set_spread_cfg(self._ctx, int(cfg)), "cs_set_spread_cfg")

    def set_sketch_dist(self, dist):
        """Distribution of the sketch's random block: "rademacher" or
        "gaussian" (variance 1/S), for later sketch_build / recon_run calls."""
        self._check(self.lib.cs_set_sketch_dist(
            self._ctx, {"rademacher": CS_SKETCH_RADEMACHER, "gaussian": CS_SKETCH_GAUSSIAN}[dist]),
            "cs_set_sketch_dist")

    def set_interp_cfg(self, cfg):
        """Select the interpolation variant: 0 global-memory gather, 1 LDS
        tiles of at most 8 coils (the default), 2 and 3 LDS tiles of at most 12
        and 4 coils."""
        self._check(self.lib.cs_set_interp_cfg(self._ctx, int(cfg)), "cs_set_interp_cfg")

    def autotune_spread(self, maps, reps=3):
        """Time every spreading shape on a normal apply with `maps` and keep
        the fastest; returns (shape index, per-shape ms per apply)."""
        ncoil = self._maps(maps)
        best = ctypes.c_int()
        ms = (ctypes.c_double * SPREAD_NCFG)()
        self._check(self.lib.cs_autotune_spread(self._ctx, _ptr(maps), ncoil, int(reps),
                                                ctypes.byref(best),
                                                ctypes.cast(ms, ctypes.c_void_p)),
                    "cs_autotune_spread")
        return best.value, list(ms)


class CNN:
    """The learned warm-start network (parameters on the device)."""

    def __init__(self, seed=0, stream=None):
        self.lib = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._n = ctypes.c_void_p()
        rc = self.lib.cs_cnn_create(ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.c_uint64(int(seed)), ctypes.byref(self._n))
        if rc != 0:
            raise CSError(f"cs_cnn_create failed ({rc})")

    def _check(self, rc, what):
        if rc != 0:
            raise CSError(f"{what} failed ({rc}): {self.lib.cs_cnn_last_error(self._n).decode()}")

    @property
    def num_params(self):
        return int(self.lib.cs_cnn_num_params(self._n))

    def get_params(self):
        import numpy as np
        p = np.empty(self.num_params, dtype=np.float32)
        self._check(self.lib.cs_cnn_get_params(self._n, p.ctypes.data, None), "get_params")
        return p

    def get_grads(self):
        import numpy as np
        g = np.empty(self.num_params, dtype=np.float32)
        self._check(self.lib.cs_cnn_get_params(self._n, None, g.ctypes.data), "get_grads")
        return g

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError("parameter count")
        self._check(self.lib.cs_cnn_set_params(self._n, p.ctypes.data), "set_params")

    @staticmethod
    def _vol(t, ch, name):
        _need(t, torch.float32, None, name)
        if t.dim() != 4 or t.shape[-1] != ch:
            raise ValueError(f"{name} must be [nz, ny, nx, {ch}]")
        return t.shape[0], t.shape[1], t.shape[2]

    def forward(self, inp):
        nz, ny, nx = self._vol(inp, 4, "inp")
        out = torch.empty((nz, ny, nx, 2), dtype=torch.float32, device=inp.device)
        self._check(self.lib.cs_cnn_forward(self._n, _ptr(inp), nz, ny, nx, _ptr(out)), "forward")
        return out

    def loss_grad(self, inp, target):
        nz, ny, nx = self._vol(inp, 4, "inp")
        if tuple(self._vol(target, 2, "target")) != (nz, ny, nx):
            raise ValueError("target shape")
        loss = ctypes.c_double()
        self._check(self.lib.cs_cnn_loss_grad(self._n, _ptr(inp), _ptr(target), nz, ny, nx,
                                              ctypes.byref(loss)), "loss_grad")
        return loss.value

    def train_step(self, inp, target, lr):
        nz, ny, nx = self._vol(inp, 4, "inp")
        if tuple(self._vol(target, 2, "target")) != (nz, ny, nx):
            raise ValueError("target shape")
        loss = ctypes.c_double()
        self._check(self.lib.cs_cnn_train_step(self._n, _ptr(inp), _ptr(target), nz, ny, nx,
                                               ctypes.c_float(lr), ctypes.byref(loss)),
                    "train_step")
        return loss.value

    def close(self):
        if getattr(self, "_n", None) and self._n.value:
            self.lib.cs_cnn_destroy(self._n)
            self._n = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent slices (one Context each, on their own streams) run
    Algorithm 1 together; the inner iterations of all slices form one HIP
    graph on the batch stream (`stream`, or one the library creates)."""

    def __init__(self, contexts, stream=None):
        self.lib = load()
        self.ctxs = list(contexts)
        # stream None: the library creates a stream of its own for the batch
        self.stream = stream
        arr = (ctypes.c_void_p * len(self.ctxs))(*[c._ctx.value for c in self.ctxs])
        self._b = ctypes.c_void_p()
        rc = self.lib.cs_batch_create(arr, len(self.ctxs),
                                      None if stream is None
                                      else ctypes.c_void_p(stream.cuda_stream),
                                      ctypes.byref(self._b))
        if rc != 0:
            raise CSError(f"cs_batch_create failed ({rc})")

    def recon(self, ys, xs, lam, T, K, V, S, seed, t0=1, step=None, n_pow=30,
              use_graph=True):
        """Run Algorithm 1 on every slice: ys[i] data, xs[i] image (in/out);
        lam, V, S, seed, step may be per-slice sequences.  Returns one dict of
        statistics per slice."""
        n = len(self.ctxs)
        per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * n
        lam, V, S, seed = per(lam), per(V), per(S), per(seed)
        step = per(0.0 if step is None else step)
        P = (ReconParams * n)()
        for i, c in enumerate(self.ctxs):
            c._data(ys[i], c.C)
            c._img(xs[i], "x")
            P[i].mode = CS_RECON_SKETCH
            P[i].lam = float(lam[i])
            P[i].T, P[i].K, P[i].V, P[i].S = int(T), int(K), int(V[i]), int(S[i])
            P[i].seed = int(seed[i])
            P[i].t0 = int(t0)
            P[i].step = float(step[i])
            P[i].n_pow = int(n_pow)
        yp = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        st = (BatchStats * n)()
        rc = self.lib.cs_batch_recon(self._b, yp, P, xp, int(bool(use_graph)), st)
        if rc != 0:
            raise CSError(f"cs_batch_recon failed ({rc}): "
                          f"{self.lib.cs_batch_last_error(self._b).decode()}")
        return [{f: getattr(s, f) for f, _ in BatchStats._fields_} for s in st]

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            self.lib.cs_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
