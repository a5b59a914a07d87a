#!/usr/bin/env python3
"""Benchmark of the coil-sketching hot path on one MI355X.

Workload: the 3D cones-like reconstruction -- 192x192x128 complex64 volume,
18000 readouts x 512 samples (9.216 M samples per coil), 32 coils, KB width 4,
oversampling 1.25 (grid 240x240x160), sketch 6 PCA + 6 Rademacher coils.  All
inputs are seeded synthetic stand-ins for the paper's 3D cones acquisitions.

One step is one outer iteration of Algorithm 1 (Sec. 2.3.4): the full-coil
gradient A^H(A x^t - y), the draw and mixing of the sketched maps, and K = 5
FISTA iterations on the sketched subproblem, each with one sketched normal
apply A_S^H A_S and one db4 wavelet prox.

Reported value: normal_apply throughput in GB/s of modelled bytes -- the
model counts, per coil, the map reads, every FFT pass reading and writing its
grid, the gridding stage reading and writing the oversampled grid, plus the
image in/out and the trajectory once -- divided by the GPU time of the
sketched normal applies measured with HIP events inside the timed steps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("normal_apply GB/s & %roofline; time-to-1e-3 NRMSE sketched+learned vs "
          "full-coil")


def model_bytes_normal(geom, ncoil):
    """Modelled HBM bytes of one normal apply with `ncoil` coils (3D NUFFT)."""
    nz, ny, nx, mz, my, mx, N = geom
    D, M = nz * ny * nx, mz * my * mx
    per_coil = 8 * (2 * D + 4 * mz * ny * nx + 4 * mz * my * nx + 4 * M)
    return ncoil * per_coil + 2 * 8 * D + 16 * N


def min_bytes_normal(D, N, ndim, ncoil):
    """Compulsory HBM bytes of one normal apply: x read and the result
    written once, each coil map read twice (the FFT between the forward and
    the adjoint multiply is a global dependency), the coordinates and the
    density weights read once (complex64 = 8 B, float32 = 4 B)."""
    return 8 * (2 * D + 2 * ncoil * D) + 4 * (ndim + 1) * N


def model_bytes_normal_2d(ny, nx, my, mx, N, ncoil):
    """Modelled HBM bytes of one 2D NUFFT normal apply: per coil the maps
    twice, one write and read of the intermediate grid per axis pass (the
    first pass pads one axis, my x nx; the second writes the my x mx grid),
    the interpolation read and the spreading write of the grid; plus x, the
    result and the coordinates and weights."""
    D, M = ny * nx, my * mx
    return ncoil * 8 * (2 * D + 4 * my * nx + 4 * M) + 2 * 8 * D + 12 * N


def hbm_copy_bandwidth(nbytes=2 << 30, reps=10):
    """Achievable HBM bandwidth of a plain device-to-device copy (bytes read
    plus bytes written, over the mean of `reps` copies)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "GB/s": 2 * nbytes / (ms * 1e-3) / 1e9}


KERNEL_LAUNCHES_PER_APPLY = {"fft_pass": 6}


def kernel_bytes(geom, cb):
    """Algorithmic bytes per launch of the main kernels for a coil chunk cb,
    split from the per-apply pass model: the six FFT passes read and write
    their grids (x and the result once per apply); the gridding stage reads
    the oversampled grid (interpolation, which also reads the 16-byte
    trajectory and weight of every sample) and writes it (spreading).  The
    sample values that pass from the interpolation to the spreading through
    HBM are not algorithmic: a fused stage keeps them on chip."""
    nz, ny, nx, mz, my, mx, N = geom
    D, M = nz * ny * nx, mz * my * mx
    passes = 8 * (cb * (2 * D + 4 * mz * ny * nx + 4 * mz * my * nx + 2 * M) + 2 * D)
    interp = 8 * M * cb + 16 * N
    spread = 8 * M * cb
    return {"fft_pass": passes / 6.0, "interp": interp, "spread": spread}


def _oracle_coil_worker(tmpdir, coils, barrier, queue):
    """One process of the CPU baseline: the oracle's normal apply for the
    given coils of the sketched map set, single-threaded, timed from a
    barrier shared by all workers (the plan is built before it)."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import nufft
    coords = np.load(os.path.join(tmpdir, "coords.npy")).astype(np.float64)
    dcf = np.load(os.path.join(tmpdir, "dcf.npy")).astype(np.float64)
    x = np.load(os.path.join(tmpdir, "x.npy")).astype(np.complex128)
    maps = np.load(os.path.join(tmpdir, "maps.npy"), mmap_mode="r")
    shape = x.shape
    plan = nufft.Plan(shape, coords, dcf)
    mine = [np.ascontiguousarray(maps[..., c:c + 1]).astype(np.complex128) for c in coils]
    barrier.wait()
    t0 = time.time()
    outs = [plan.normal(x, m) for m in mine]
    t1 = time.time()
    queue.put((coils, t0, t1, outs[0] if 0 in coils else None))


def cpu_baseline(p, Ch, geom, max_workers=16):
    """The FP64 oracle, as it stands, on one complete sketched normal apply at
    full size: the Ch coils are independent, so each runs in its own
    single-threaded worker process (NumPy's FFT and bincount are
    single-threaded) on up to min(Ch, cores, max_workers) host cores.  The
    time is the span from the common start barrier to the last worker's end.
    Returns the baseline record and the oracle's result for the first coil
    (the FP64 reference of the precision report)."""
    import multiprocessing as mp
    import shutil
    import tempfile
    import numpy as np
    workers = max(1, min(Ch, os.cpu_count() or 1, max_workers))
    groups = [list(range(w, Ch, workers)) for w in range(workers)]
    tmp = tempfile.mkdtemp(prefix="cs_cpu_baseline_")
    try:
        np.save(os.path.join(tmp, "coords.npy"), p.coords.astype(np.float32))
        np.save(os.path.join(tmp, "dcf.npy"), p.dcf.astype(np.float32))
        np.save(os.path.join(tmp, "x.npy"), p.x_true.astype(np.complex64))
        # stand-in for the Ch sketched maps: the first Ch coil maps (the cost
        # does not depend on the values)
        np.save(os.path.join(tmp, "maps.npy"),
                np.ascontiguousarray(p.maps[..., :Ch]).astype(np.complex64))
        ctx = mp.get_context("spawn")
        barrier, queue = ctx.Barrier(workers), ctx.Queue()
        procs = [ctx.Process(target=_oracle_coil_worker, args=(tmp, g, barrier, queue))
                 for g in groups]
        for pr in procs:
            pr.start()
        res = [queue.get() for _ in procs]
        for pr in procs:
            pr.join()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    t0 = min(r[1] for r in res)
    t1 = max(r[2] for r in res)
    ref = next(r[3] for r in res if r[3] is not None)
    secs = t1 - t0
    gbs = model_bytes_normal(geom, Ch) / secs / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": (f"one {Ch}-coil sketched normal apply at full size "
                       f"({p.shape[0]}x{p.shape[1]}x{p.shape[2]}, {p.coords.shape[0]} "
                       f"samples), one coil per single-threaded worker, {secs:.1f} s"),
            "seconds_per_apply": round(secs, 2)}, ref


TTA_THRESHOLDS = (5e-2, 1e-2, 1e-3)


def first_below(dist, thr):
    for i, d in enumerate(dist):
        if d <= thr:
            return i
    return None


def image_quality(x, ref, sigma=1.5):
    """NRMSE, SSIM and HFEN of the magnitude image |x| against |ref| (the
    metrics of Sec. 3.2.1 / 3.3.1, computed against the synthetic phantom).
    SSIM (Wang et al. 2004): Gaussian window of width sigma, K1 = 0.01,
    K2 = 0.03, dynamic range max |ref|, averaged over the image.  HFEN
    (Ravishankar and Bresler 2011): relative l2 error of the
    Laplacian-of-Gaussian (width sigma) filtered images."""
    import numpy as np
    from scipy import ndimage
    a = np.abs(np.asarray(x, dtype=np.complex128))
    r = np.abs(np.asarray(ref, dtype=np.complex128))
    L = r.max()
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    g = lambda v: ndimage.gaussian_filter(v, sigma, mode="wrap")
    ma, mr = g(a), g(r)
    va, vr, cov = g(a * a) - ma * ma, g(r * r) - mr * mr, g(a * r) - ma * mr
    ssim = ((2 * ma * mr + c1) * (2 * cov + c2)) / ((ma * ma + mr * mr + c1) * (va + vr + c2))
    la = ndimage.gaussian_laplace(a, sigma, mode="wrap")
    lr = ndimage.gaussian_laplace(r, sigma, mode="wrap")
    return {"nrmse": float(np.linalg.norm(a - r) / np.linalg.norm(r)),
            "ssim": float(np.mean(ssim)),
            "hfen": float(np.linalg.norm(la - lr) / np.linalg.norm(lr))}


def reference_minimizer(ctx, y, p, lam, log, outer=40, K=100, polish_chunk=500,
                        polish_max=6000, tol=1e-6):
    """x_inf for the time-to-accuracy runs: the full-coil problem's minimizer.
    Algorithm 1 converges linearly to it (its subproblems keep the true
    gradient, and a subproblem started at the minimizer stays there however
    few inner iterations it runs), so `outer` outer iterations with K = 100
    inner FISTA iterations (V = C^ - 1, S = 1) come within FP32 rounding of
    it; full-coil FISTA then polishes in chunks of `polish_chunk` iterations
    (momentum restarted per chunk) until a chunk changes x by less than tol
    relative.  Returns x_inf and a record of how it was reached."""
    import torch
    t0 = time.time()
    Ch = p.V + p.S
    x = torch.zeros(p.shape, dtype=torch.complex64, device=y.device)
    changes = []
    for it in range(outer):
        prev = x.clone()
        ctx.recon_run(y, mode="sketch", lam=lam, T=1, K=K, V=Ch - 1, S=1, seed=p.seed + 101,
                      t0=it + 1, step=0.0, n_pow=30, reuse_b=it > 0, x=x)
        changes.append((torch.linalg.vector_norm(x - prev) /
                        torch.linalg.vector_norm(x)).item())
    log(f"{p.name} x_inf: {outer} outer iterations of Algorithm 1 (K={K}), last change "
        f"{changes[-1]:.3e}")
    pf = ctx.recon_run(y, mode="full", lam=lam, T=0, step=0.0, n_pow=30)
    its, change = 0, None
    while its < polish_max:
        prev = x.clone()
        ctx.recon_run(y, mode="full", lam=lam, T=polish_chunk, step=pf.alpha, reuse_b=True, x=x)
        its += polish_chunk
        change = (torch.linalg.vector_norm(x - prev) / torch.linalg.vector_norm(x)).item()
        log(f"{p.name} x_inf: polish {its} full-coil FISTA iterations, chunk change {change:.3e}")
        if change < tol:
            break
    return x, {"method": "Algorithm 1 then full-coil FISTA polish", "alg1_outer": outer,
               "alg1_K": K, "alg1_changes_last5": changes[-5:], "polish_iterations": its,
               "polish_chunk": polish_chunk, "last_chunk_rel_change": change,
               "wall_s": round(time.time() - t0, 1)}


def time_to_accuracy(ctx, y, p, args, log, ref_iters, full_iters, outer_iters, chunk,
                     cnn=None, lam=None, restart=0, x_ref=None, sketch_seeds=1):
    """Time to d(x^t) = ||x^t - x_inf|| / ||x_inf|| <= thr (Sec. 3.3.1) for the
    plain full-coil FISTA and for Algorithm 1, both in FP32 on this GPU, at
    the paper's 5% criterion and at 1e-2 and 1e-3.

    x_inf is the full-coil problem's minimizer, found by plain FISTA run in
    chunks (momentum restarted per chunk) until one chunk changes x by less
    than 1e-6 relative, or ref_iters iterations.  Times are GPU event times on
    the context stream: `loop_ms` covers the iterations up to the first one
    within the threshold, `total_ms` adds the set-up (b = A^H y, step size by
    power iteration, PCA basis and first sketch)."""
    import numpy as np
    import torch
    lam = p.lam if lam is None else lam
    C, V, S = p.n_coils, p.V, p.S
    dev = y.device
    t0 = time.time()
    pf = ctx.recon_run(y, mode="full", lam=lam, T=0, step=0.0, n_pow=30)
    alpha_f = pf.alpha
    x_inf = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
    change, its = None, 0
    if x_ref is not None:
        x_inf, ref = x_ref
        ref_iters = 0
    while its < ref_iters:
        prev = x_inf.clone()
        ctx.recon_run(y, mode="full", lam=lam, T=chunk, step=alpha_f, reuse_b=True, x=x_inf)
        its += chunk
        change = (torch.linalg.vector_norm(x_inf - prev) /
                  torch.linalg.vector_norm(x_inf)).item()
        if its % (chunk * 5) == 0 or change < 1e-6:
            log(f"{p.name} x_inf: {its} full FISTA iterations, last-chunk change {change:.3e}")
        if change < 1e-6:
            break
    if x_ref is None:
        ref = {"iterations": its, "chunk": chunk, "last_chunk_rel_change": change,
               "wall_s": round(time.time() - t0, 1)}

    def summarize(r, n_full_per_it, n_sk_per_it, pre_full, pre_sk, extra_ms=0.0, ch=V + S):
        out = {"prep_ms": r.prep_ms + extra_ms, "iterations_run": len(r.dist),
               "final_dist": r.dist[-1] if r.dist else None, "alpha": r.alpha,
               "ms_per_iteration": r.time_ms[-1] / max(1, len(r.time_ms))}
        for thr in TTA_THRESHOLDS:
            i = first_below(r.dist, thr)
            key = f"{thr:g}"
            if i is None:
                out[key] = None
                continue
            fa = pre_full + (i + 1) * n_full_per_it
            sa = pre_sk + (i + 1) * n_sk_per_it
            out[key] = {"iterations": i + 1, "loop_ms": r.time_ms[i],
                        "total_ms": r.time_ms[i] + r.prep_ms + extra_ms,
                        "full_applies": fa, "sketched_applies": sa,
                        "coil_ffts": 2 * (fa * C + sa * ch)}
        return out

    x = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
    rf = ctx.recon_run(y, mode="full", lam=lam, T=full_iters, step=0.0, n_pow=30,
                       reuse_b=False, x=x, x_ref=x_inf)
    full = summarize(rf, 1, 0, 31, 0)
    full["image_quality"] = image_quality(rf.x.cpu().numpy(), p.x_true)
    log(f"{p.name} full-coil FISTA: final d {full['final_dist']:.3e}, "
        + ", ".join(f"{k}: {v and round(v['total_ms'], 1)} ms" for k, v in full.items()
                    if k in {f'{t:g}' for t in TTA_THRESHOLDS}))
    # the same with momentum restarted every `restart` iterations, as the
    # inner solves of Algorithm 1 restart it at every subproblem
    restart_runs = {}
    if restart:
        x = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
        r0 = ctx.recon_run(y, mode="full", lam=lam, T=0, step=0.0, n_pow=30, x=x)
        dist, tms, off = [], [], 0.0
        for _ in range(max(1, full_iters // restart)):
            r = ctx.recon_run(y, mode="full", lam=lam, T=restart, step=r0.alpha, reuse_b=True,
                              x=x, x_ref=x_inf)
            dist += list(r.dist)
            tms += [off + t for t in r.time_ms]
            off = tms[-1]
        rr = SimpleNamespace(prep_ms=r0.prep_ms, dist=dist, time_ms=tms, alpha=r0.alpha)
        fr = summarize(rr, 1, 0, 31, 0)
        fr["restart_every"] = restart
        log(f"{p.name} full-coil FISTA restarted every {restart}: final d "
            f"{fr['final_dist']:.3e}, "
            + ", ".join(f"{k}: {v and round(v['total_ms'], 1)} ms" for k, v in fr.items()
                        if k in {f'{t:g}' for t in TTA_THRESHOLDS}))
        restart_runs[f"full_coil_restart{restart}"] = fr

    # PCA basis recomputed so that its cost is part of the sketched set-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    ctx.sketch_build(y, V, S, p.seed, 1, refresh=True, host_outputs=False)
    ev[1].record()
    torch.cuda.synchronize()
    pca_ms = ev[0].elapsed_time(ev[1])
    res = {"lam": lam, "x_inf": ref, "full_coil": full, **restart_runs}
    # inner iterations K per subproblem are not fixed by the paper: report
    # several.  runs: (label, K, outer iterations, mode[, V, S]); V and S
    # default to the problem's sketch
    for run, sseed in ((r, k) for r in outer_iters for k in range(sketch_seeds)):
        label, K, T, mode = run[:4]
        rV, rS = run[4:6] if len(run) > 4 else (V, S)
        if mode == "learned" and cnn is None:
            continue
        x = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
        rs = ctx.recon_run(y, mode=mode, lam=lam, T=T, K=K, V=rV, S=rS, seed=p.seed + sseed,
                           t0=1, step=0.0, n_pow=30, reuse_b=False, x=x, x_ref=x_inf, cnn=cnn)
        # the learned mode's decision applies one extra sketched operator
        sk = summarize(rs, 1, K + (1 if mode == "learned" else 0), 0, 31, extra_ms=pca_ms,
                       ch=rV + rS)
        sk["V"], sk["S"] = rV, rS
        if mode == "learned":
            sk["warm_accepted"] = rs.n_warm_accepted
            sk["warm_rejected"] = rs.n_warm_rejected
            sk["ms_warm_decisions"] = rs.ms_warm
        log(f"{p.name} {label} (K={K}, V={rV}, S={rS}): final d {sk['final_dist']:.3e}, "
            + ", ".join(f"{k}: {v and round(v['total_ms'], 1)} ms" for k, v in sk.items()
                        if k in {f'{t:g}' for t in TTA_THRESHOLDS}))
        sk["speedup_total"] = {}
        for thr in TTA_THRESHOLDS:
            k = f"{thr:g}"
            if full.get(k) and sk.get(k):
                sk["speedup_total"][k] = full[k]["total_ms"] / sk[k]["total_ms"]
        for name, fr in restart_runs.items():
            sk[f"speedup_vs_{name}"] = {f"{t:g}": fr[f"{t:g}"]["total_ms"] / sk[f"{t:g}"]["total_ms"]
                                        for t in TTA_THRESHOLDS
                                        if fr.get(f"{t:g}") and sk.get(f"{t:g}")}
        sk["image_quality"] = image_quality(rs.x.cpu().numpy(), p.x_true)
        sk["sketch_seed"] = p.seed + sseed
        name = f"{label}_K{K}" + ("" if (rV, rS) == (V, S) else f"_V{rV}S{rS}")
        if sketch_seeds > 1:
            name += f"_seed{sseed}"
        res[name] = sk
    if sketch_seeds > 1:
        # median and range over the sketch seeds of each run's speed-up
        summary = {}
        for run in outer_iters:
            label, K = run[0], run[1]
            rV, rS = run[4:6] if len(run) > 4 else (V, S)
            base = f"{label}_K{K}" + ("" if (rV, rS) == (V, S) else f"_V{rV}S{rS}")
            per = [res.get(f"{base}_seed{k}") for k in range(sketch_seeds)]
            per = [r for r in per if r]
            if not per:
                continue
            summary[base] = {}
            for thr in TTA_THRESHOLDS:
                k = f"{thr:g}"
                ms = [r[k]["total_ms"] for r in per if r.get(k)]
                sp = [r["speedup_total"].get(k) for r in per if r["speedup_total"].get(k)]
                summary[base][k] = {"reached": f"{len(ms)}/{len(per)}",
                                    "total_ms_median": float(np.median(ms)) if ms else None,
                                    "speedup_median": float(np.median(sp)) if sp else None,
                                    "speedup_range": [min(sp), max(sp)] if sp else None}
        res["over_sketch_seeds"] = summary
    return res


def train_warm_start(args, log, n_problems=6, T=8, K=100, steps=600, lam=5e-4, V=7, S=1):
    """The warm-start network, trained on solver pairs from small cones
    problems (32^3, 16 coils, sketch V+S, K inner iterations, regularisation
    weight lam) with the library's MFMA kernels."""
    import numpy as np
    import torch
    import synth
    from paper_2305_06482_amd import CNN, Context, learned
    t0 = time.time()
    probs = []
    for i in range(n_problems):
        p = synth.make_cones(shape=(32, 32, 32), n_readouts=600, n_samples=96, n_coils=16,
                             V=V, S=S, seed_base=7000 + 10 * i, lam=lam)
        ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0], wav_levels=3)
        maps = torch.from_numpy(p.maps).to(torch.complex64).cuda()
        dcf = torch.from_numpy(p.dcf).to(torch.float32).cuda()
        ctx.set_operator(maps, coords=torch.from_numpy(p.coords).to(torch.float32).cuda(),
                         dcf=dcf)
        y = ctx.sense_apply(maps, torch.from_numpy(p.x_true).to(torch.complex64).cuda())
        y += torch.from_numpy(p.noise).to(torch.complex64).cuda() * \
            dcf.sqrt()[:, None].to(torch.complex64)
        probs.append((ctx, y, p.V, p.S, p.seed, p.lam))
    ins, tgts = learned.collect_pairs(probs, T, K)
    net = CNN(seed=1)
    t1 = time.time()
    losses = learned.train(net, ins, tgts, steps, patch=(32, 32, 32), lr=1e-3)
    torch.cuda.synchronize()
    for c, *_ in probs:
        c.close()
    info = {"problems": n_problems, "pairs": len(ins), "steps": steps, "K": K, "V": V, "S": S,
            "lam": lam,
            "loss_first": float(np.mean(losses[:20])), "loss_last": float(np.mean(losses[-20:])),
            "train_s": round(time.time() - t1, 2), "total_s": round(time.time() - t0, 1)}
    log(f"warm-start network trained: {info}")
    return net, info


def cartesian_tta(p, args, log, outer_iters=None):
    """Time to accuracy on a Cartesian problem (its own context)."""
    import numpy as np
    import torch
    from paper_2305_06482_amd import Context
    dev = torch.device("cuda:0")
    dt = lambda a, d: torch.from_numpy(np.ascontiguousarray(a)).to(d).to(dev)
    C = p.n_coils
    ctx = Context(p.shape, C, "cart", wav_levels=4)
    maps = dt(p.maps, torch.complex64)
    mask = dt(p.mask, torch.uint8)
    ctx.set_operator(maps, mask=mask)
    y = ctx.sense_apply(maps, dt(p.x_true, torch.complex64))
    y += dt(p.noise.reshape(p.shape + (C,)), torch.complex64) * mask[..., None]
    if outer_iters is None:
        outer_iters = [("sketched", 5, 800, "sketch"),
                       ("sketched", 20, 250, "sketch"),
                       ("sketched", 20, 250, "sketch", p.V + p.S - 1, 1)]
    res = time_to_accuracy(ctx, y, p, args, log, ref_iters=20000, full_iters=4000,
                           outer_iters=outer_iters, chunk=1000)
    ctx.close()
    return res


def cartesian_tta_seeds(first, args, log, seeds):
    """Time to accuracy on the 320 x 320 Cartesian problem over `seeds`
    independent draws of phantom, maps, mask, noise and sketch seed (the
    first is the run `first`, the others use held-out seed bases): full-coil
    FISTA against Algorithm 1 with K = 20, V = C^ - 1, S = 1.  Reports the
    times per draw and the median and range of the speed-up."""
    import numpy as np
    import synth

    def pick(r):
        return r["full_coil"], next(v for k, v in r.items()
                                    if k.startswith("sketched_K20_V") and k.endswith("S1"))
    runs = [pick(first)]
    bases = [2000]
    for k in range(1, seeds):
        base = 2000 + 100 * k
        pc = synth.make_cart_clinical(seed_base=base)
        r = cartesian_tta(pc, args, log, outer_iters=[("sketched", 20, 250, "sketch",
                                                       pc.V + pc.S - 1, 1)])
        runs.append(pick(r))
        bases.append(base)
    out = {"seed_bases": bases}
    for thr in TTA_THRESHOLDS:
        key = f"{thr:g}"
        f = [a[key]["total_ms"] if a[key] else None for a, _ in runs]
        s = [b[key]["total_ms"] if b[key] else None for _, b in runs]
        ratio = [fa / sa for fa, sa in zip(f, s) if fa is not None and sa is not None]
        out[key] = {"full_ms": f, "sketched_ms": s, "both_reached": len(ratio),
                    "speedup_median": float(np.median(ratio)) if ratio else None,
                    "speedup_min": min(ratio) if ratio else None,
                    "speedup_max": max(ratio) if ratio else None}
    log("cart320 over seeds: " + ", ".join(
        f"{k}: speed-up median {v['speedup_median'] and round(v['speedup_median'], 2)} "
        f"[{v['speedup_min'] and round(v['speedup_min'], 2)}, "
        f"{v['speedup_max'] and round(v['speedup_max'], 2)}] ({v['both_reached']} reached)"
        for k, v in out.items() if k != "seed_bases"))
    return out


def gfactor_bench(args, log, n=256, C=8, accel=3, trials=60, lam=1e-2, sigma=1e-2,
                  T_full=60, T=10, K=20, designs=((3, 1), (2, 2)), seed=8000):
    """Monte-Carlo inverse g-factor of l2 reconstructions (Sec. 3.2.2):
    regular R = 3 Cartesian sampling, `trials` noise realisations, full-coil
    CG against Algorithm 1 with CG inner solves.  g = sd_R / (sd_full sqrt(R))
    per pixel, sd_full from fully sampled reconstructions of the same noise
    level; the sketch design (PCA basis) is fixed by the first trial, so every
    reconstruction is the same linear map of the data."""
    import numpy as np
    import torch
    import synth
    from paper_2305_06482_amd import Context
    dev = torch.device("cuda:0")
    t0 = time.time()
    shape = (n, n)
    x = torch.from_numpy(synth.phantom(shape, seed)).to(torch.complex64).to(dev)
    maps = torch.from_numpy(synth.coil_maps(shape, C, seed + 1)).to(torch.complex64).to(dev)
    mask_u = synth.mask_regular(n, n, accel=accel)
    R = mask_u.size / mask_u.sum()
    ctxs = {}
    for name, mk in (("under", mask_u), ("full", np.ones(shape, np.uint8))):
        c = Context(shape, C, "cart", wav_levels=4)
        c.set_operator(maps, mask=torch.from_numpy(mk).to(dev))
        ctxs[name] = (c, torch.from_numpy(mk).to(torch.float32).to(dev)[..., None],
                      c.sense_apply(maps, x))
    gen = torch.Generator(device=dev).manual_seed(seed)
    runs = {"full_coil": None, **{f"sketch_V{V}S{S}": (V, S) for V, S in designs}}
    acc = {k: [torch.zeros(shape, dtype=torch.complex128, device=dev),
               torch.zeros(shape, dtype=torch.float64, device=dev), 0.0] for k in runs}
    acc["fully_sampled"] = [torch.zeros(shape, dtype=torch.complex128, device=dev),
                            torch.zeros(shape, dtype=torch.float64, device=dev), 0.0]

    def add(key, xr, ms):
        a = acc[key]
        a[0] += xr.to(torch.complex128)
        a[1] += xr.abs().to(torch.float64) ** 2
        a[2] += ms

    for tr in range(trials):
        for name in ("under", "full"):
            c, m, y0 = ctxs[name]
            nz = torch.randn(shape + (C, 2), generator=gen, device=dev) * (sigma / math.sqrt(2))
            y = y0 + torch.view_as_complex(nz.contiguous()) * m
            if name == "full":
                r = c.recon_run(y, mode="full", reg="l2", lam=lam, T=T_full)
                add("fully_sampled", r.x, r.total_ms)
                continue
            for key, vs in runs.items():
                if vs is None:
                    r = c.recon_run(y, mode="full", reg="l2", lam=lam, T=T_full)
                else:
                    r = c.recon_run(y, mode="sketch", reg="l2", lam=lam, T=T, K=K, V=vs[0],
                                    S=vs[1], seed=seed)
                add(key, r.x, r.total_ms + r.prep_ms)
    torch.cuda.synchronize()

    def sd(key):
        a = acc[key]
        mean = a[0] / trials
        return ((a[1] / trials - mean.abs() ** 2).clamp_min(0) * trials / (trials - 1)).sqrt()

    support = x.abs() > 0.05 * x.abs().max()
    sd_ref = sd("fully_sampled")
    res = {"shape": list(shape), "coils": C, "R": round(float(R), 3), "trials": trials,
           "lam": lam, "sigma": sigma, "T_full": T_full, "T": T, "K": K}
    for key in runs:
        inv = (sd_ref * math.sqrt(R) / sd(key))[support].cpu().numpy()
        res[key] = {"inv_g_mean": float(np.mean(inv)), "inv_g_p5": float(np.percentile(inv, 5)),
                    "inv_g_min": float(np.min(inv)),
                    "ms_per_recon": acc[key][2] / trials}
    res["wall_s"] = round(time.time() - t0, 1)
    for c, *_ in ctxs.values():
        c.close()
    log(f"inverse g-factor ({trials} trials, {n}x{n}, {C} coils, R={R:.2f}): " +
        ", ".join(f"{k}: mean {v['inv_g_mean']:.3f} p5 {v['inv_g_p5']:.3f}, "
                  f"{v['ms_per_recon']:.2f} ms" for k, v in res.items() if isinstance(v, dict)))
    return res


def tv_tta(args, log, lam=5e-3, n_cg=3, ref_iters=3000, full_iters=400,
           runs=((20, 60, 11, 1), (50, 24, 11, 1), (20, 60, 6, 6)), seed=3000):
    """l1-TV (Sec. 3.3.2) time to accuracy on the 48^3 cones instance
    (32 coils): PDHG with n_cg CG iterations per data-consistency step,
    full-coil against Algorithm 1 with K PDHG iterations per subproblem.
    x_inf = ref_iters full-coil PDHG iterations.  Times are GPU event times
    plus set-up."""
    import numpy as np
    import torch
    import synth
    from paper_2305_06482_amd import Context
    dev = torch.device("cuda:0")
    t0 = time.time()
    p = synth.make_cones_small(seed_base=seed)
    ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0], wav_levels=3)
    maps = torch.from_numpy(p.maps).to(torch.complex64).to(dev)
    w = torch.from_numpy(p.dcf).to(torch.float32).to(dev)
    ctx.set_operator(maps, coords=torch.from_numpy(p.coords).to(torch.float32).to(dev), dcf=w)
    y = ctx.sense_apply(maps, torch.from_numpy(p.x_true).to(torch.complex64).to(dev))
    y += torch.from_numpy(p.noise).to(torch.complex64).to(dev) * w.sqrt()[:, None].to(torch.complex64)
    x_inf = ctx.recon_run(y, mode="full", reg="tv", lam=lam, T=ref_iters, n_cg=n_cg).x

    def times(r):
        out = {"final_dist": r.dist[-1], "prep_ms": r.prep_ms,
               "full_applies": r.n_full_applies, "sketched_applies": r.n_sketch_applies}
        for thr in TTA_THRESHOLDS:
            i = first_below(r.dist, thr)
            out[f"{thr:g}"] = None if i is None else {
                "iterations": i + 1, "total_ms": r.time_ms[i] + r.prep_ms}
        return out

    res = {"shape": list(p.shape), "coils": p.n_coils, "lam": lam, "n_cg": n_cg,
           "x_inf_iterations": ref_iters}
    rf = ctx.recon_run(y, mode="full", reg="tv", lam=lam, T=full_iters, n_cg=n_cg, x_ref=x_inf)
    res["full_coil"] = times(rf)
    for K, T, V, S in runs:
        r = ctx.recon_run(y, mode="sketch", reg="tv", lam=lam, T=T, K=K, V=V, S=S, seed=p.seed,
                          n_cg=n_cg, x_ref=x_inf)
        e = times(r)
        e["speedup_total"] = {k: res["full_coil"][k]["total_ms"] / e[k]["total_ms"]
                              for k in (f"{t:g}" for t in TTA_THRESHOLDS)
                              if res["full_coil"].get(k) and e.get(k)}
        res[f"sketched_K{K}_V{V}S{S}"] = e
    ctx.close()
    res["wall_s"] = round(time.time() - t0, 1)
    log("l1-TV time to accuracy (48^3 cones): " + "; ".join(
        f"{k}: " + ", ".join(f"{t}: {v[t] and round(v[t]['total_ms'], 1)} ms"
                            for t in (f"{x:g}" for x in TTA_THRESHOLDS))
        for k, v in res.items() if isinstance(v, dict) and "final_dist" in v))
    return res


def design_ablation(args, log, n=256, C=8, seeds=20, chats=(3, 4), T=10, K=10, lam=1e-3,
                    T_base=300, seed_base=8100):
    """Sketching-matrix design (Sec. 3.2.1) on a synthetic 2D radial slice
    (R = 2, 8 coils, l1-wavelet): for C^ in chats, V = 0..C^ (S = C^ - V) and
    Rademacher / Gaussian entries, `seeds` runs of Algorithm 1 with T outer
    and K inner iterations; objective and NRMSE against the phantom, each
    normalised by those of the full-coil FISTA baseline (T_base
    iterations)."""
    import numpy as np
    import torch
    import synth
    from paper_2305_06482_amd import Context, CSError
    dev = torch.device("cuda:0")
    t0 = time.time()
    shape = (n, n)
    spokes = int(round(math.pi / 2 * n / 2))  # half the Nyquist spoke count: R = 2
    coords = synth.radial_traj(n, spokes)
    dcf = synth.radial_dcf(coords, n)
    xt = torch.from_numpy(synth.phantom(shape, seed_base)).to(torch.complex64).to(dev)
    maps = torch.from_numpy(synth.coil_maps(shape, C, seed_base + 1)).to(torch.complex64).to(dev)
    ctx = Context(shape, C, "noncart", nsamp=coords.shape[0], wav_levels=4)
    w = torch.from_numpy(dcf).to(torch.float32).to(dev)
    ctx.set_operator(maps, coords=torch.from_numpy(coords).to(torch.float32).to(dev), dcf=w)
    noise = torch.from_numpy(synth.complex_noise((coords.shape[0], C), 1e-3, seed_base + 2))
    y = ctx.sense_apply(maps, xt) + noise.to(torch.complex64).to(dev) * \
        w.sqrt()[:, None].to(torch.complex64)

    def metrics(x):
        r = ctx.sense_apply(maps, x) - y
        obj = 0.5 * float((r.abs().double() ** 2).sum()) + \
            lam * float(ctx.dwt(x).abs().double().sum())
        nr = float((x - xt).abs().double().norm() / xt.abs().double().norm())
        return obj, nr

    base = ctx.recon_run(y, mode="full", lam=lam, T=T_base)
    f0, e0 = metrics(base.x)
    res = {"shape": list(shape), "coils": C, "spokes": spokes, "seeds": seeds, "T": T, "K": K,
           "lam": lam, "baseline": {"objective": f0, "nrmse": e0, "iterations": T_base}}
    for ch in chats:
        for V in range(ch + 1):
            S = ch - V
            for dist in (("rademacher", "gaussian") if S > 0 else ("none",)):
                if dist != "none":
                    ctx.set_sketch_dist(dist)
                fs, es, diverged = [], [], 0
                runs = seeds if S > 0 else 1
                for sd in range(runs):
                    try:
                        r = ctx.recon_run(y, mode="sketch", lam=lam, T=T, K=K, V=V, S=S,
                                          seed=seed_base + 17 * sd)
                    except CSError:  # the library stops a run whose iterate overflows
                        diverged += 1
                        continue
                    f, e = metrics(r.x)
                    if not (math.isfinite(f) and f < 1e6 * f0):
                        diverged += 1
                        continue
                    fs.append(f / f0)
                    es.append(e / e0)
                fs, es = np.array(fs), np.array(es)
                ok = fs.size > 0
                res[f"C{ch}_V{V}_S{S}_{dist}"] = {
                    "objective_rel_median": float(np.median(fs)) if ok else None,
                    "nrmse_rel_median": float(np.median(es)) if ok else None,
                    "objective_rel_mean": float(np.mean(fs)) if ok else None,
                    "objective_rel_std": float(np.std(fs)) if ok else None,
                    "nrmse_rel_mean": float(np.mean(es)) if ok else None,
                    "nrmse_rel_std": float(np.std(es)) if ok else None,
                    "runs": runs, "diverged": diverged}
    ctx.set_sketch_dist("rademacher")
    ctx.close()
    res["wall_s"] = round(time.time() - t0, 1)
    log("design ablation (objective / baseline: median, mean +- std): " + ", ".join(
        (f"{k}: median {v['objective_rel_median']:.4f}, "
         f"{v['objective_rel_mean']:.4f}+-{v['objective_rel_std']:.4f}"
         if v["objective_rel_mean"] is not None else f"{k}: diverged") +
        (f" ({v['diverged']}/{v['runs']} diverged)" if v["diverged"] else "")
        for k, v in res.items() if isinstance(v, dict) and "runs" in v))
    return res


def batched_bench(args, log, T=3, K=5):
    """The batched workload: 64 independent 2D golden-angle radial slices of
    uneven matrix size, spoke count, coil count and sketch size, each on its
    own context and stream, run together by the batch executor.  Reports the
    host wall time per outer iteration of Algorithm 1 with the inner
    iterations issued eagerly and as one replayed HIP graph (same kernels,
    bit-identical results), after tuning each geometry's spreading shape."""
    import numpy as np
    import torch
    import synth
    from paper_2305_06482_amd import Batch, Context, autotune
    t0 = time.time()
    specs = synth.batched_radial_specs()
    sl = []
    tuned = {}
    for i, s in enumerate(specs):
        p = synth.make_radial(s["n"], s["spokes"], s["coils"], s["V"], s["S"],
                              seed_base=6000 + 10 * i)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ctx = Context(p.shape, p.n_coils, "noncart", nsamp=p.coords.shape[0], wav_levels=4)
            maps = torch.from_numpy(p.maps).to(torch.complex64).cuda()
            dcf = torch.from_numpy(p.dcf).to(torch.float32).cuda()
            ctx.set_operator(maps, coords=torch.from_numpy(p.coords).to(torch.float32).cuda(),
                             dcf=dcf)
            y = ctx.sense_apply(maps, torch.from_numpy(p.x_true).to(torch.complex64).cuda())
            y += (torch.from_numpy(p.noise).to(torch.complex64).cuda()
                  * dcf.sqrt()[:, None].to(torch.complex64))
            shape, _, hit = autotune.tune(ctx, maps[..., :p.V + p.S].contiguous(), reps=2)
        tuned[shape] = tuned.get(shape, 0) + 1
        sl.append((p, ctx, maps, y))
    torch.cuda.synchronize()
    log(f"batched: {len(sl)} slices set up in {time.time() - t0:.1f} s, "
        f"spreading shapes {tuned}")
    # modelled bytes of the normal applies of one outer iteration of every
    # slice: one full-coil apply and K sketched applies
    apply_bytes = 0
    for p, ctx, _, _ in sl:
        _, my, mx = ctx.grid_shape()
        ny, nx = p.shape
        N = p.coords.shape[0]
        apply_bytes += (model_bytes_normal_2d(ny, nx, my, mx, N, p.n_coils)
                        + K * model_bytes_normal_2d(ny, nx, my, mx, N, p.V + p.S))
    res = {"slices": len(sl), "samples_per_coil_total": int(sum(p.coords.shape[0]
                                                              for p, *_ in sl)),
           "apply_model_bytes_per_outer_iteration": int(apply_bytes),
           "coil_samples_total": int(sum(p.coords.shape[0] * p.n_coils for p, *_ in sl)),
           "outer_iterations": T, "K": K, "spread_shapes": {str(k): v for k, v in tuned.items()}}
    # the applies alone, as the batched path issues them: each slice's
    # one full-coil and K sketched normal applies on its own stream, all
    # slices at once; wall time between two events that bracket every stream
    sk_maps = [ctx.sketch_build(y, p.V, p.S, p.seed, 1, host_outputs=False)[0]
               for p, ctx, _, y in sl]
    probes = [torch.randn(p.shape, dtype=torch.complex64, device="cuda") for p, *_ in sl]
    outs = [torch.empty_like(v) for v in probes]
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    walls = []
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(main)
        ends = []
        for (p, ctx, maps, _), sm, v, o in zip(sl, sk_maps, probes, outs):
            ctx.stream.wait_event(e0)
            ctx.normal_apply(maps, v, out=o)
            for _ in range(K):
                ctx.normal_apply(sm, v, out=o)
            ev = torch.cuda.Event()
            ev.record(ctx.stream)
            ends.append(ev)
        for ev in ends:
            main.wait_event(ev)
        e1.record(main)
        torch.cuda.synchronize()
        walls.append(e0.elapsed_time(e1))
    apply_ms = float(np.median(walls[1:]))
    res["applies_ms_per_outer_iteration"] = apply_ms
    res["applies_model_GBs"] = apply_bytes / (apply_ms * 1e-3) / 1e9
    res["applies_pct_hbm_roofline"] = 100 * res["applies_model_GBs"] / HBM_PEAK_GBS
    log(f"batched: the applies of one outer iteration of all slices take {apply_ms:.2f} ms, "
        f"{res['applies_model_GBs']:.0f} GB/s of modelled bytes")
    xs = {}
    for use_graph in (False, True, False, True):
        x = [torch.zeros(p.shape, dtype=torch.complex64, device="cuda") for p, *_ in sl]
        torch.cuda.synchronize()
        b = Batch([c for _, c, _, _ in sl])
        st = b.recon([y for *_, y in sl], x, [p.lam for p, *_ in sl], T, K,
                     [p.V for p, *_ in sl], [p.S for p, *_ in sl], [p.seed for p, *_ in sl],
                     use_graph=use_graph)
        b.close()
        key = "graph" if use_graph else "eager"
        res[f"{key}_ms_per_outer_iteration"] = st[0]["wall_loop_ms"] / T
        res[f"{key}_prep_ms"] = st[0]["wall_prep_ms"]
        if use_graph:
            res["graph_nodes"] = st[0]["graph_nodes"]
        xs[key] = x
    res["graph_equals_eager"] = all(torch.equal(a, b) for a, b in zip(xs["eager"], xs["graph"]))
    res["graph_speedup"] = res["eager_ms_per_outer_iteration"] / res["graph_ms_per_outer_iteration"]
    # a lower bound on the applies' bandwidth: the time also holds the prox,
    # the coil mixing and the host's launch work
    best = min(res["eager_ms_per_outer_iteration"], res["graph_ms_per_outer_iteration"])
    res["apply_model_GBs_lower_bound"] = apply_bytes / (best * 1e-3) / 1e9
    log(f"batched: eager {res['eager_ms_per_outer_iteration']:.1f} ms, graph "
        f"{res['graph_ms_per_outer_iteration']:.1f} ms per outer iteration "
        f"({res['graph_nodes']} graph nodes), identical {res['graph_equals_eager']}")
    for _, c, _, _ in sl:
        c.close()
    return res


def precision_report(ctx, p, Ch, cpu_ref, log):
    """Error of FP32 results against FP64 (oracle or host FP64 arithmetic)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    out = {}
    if cpu_ref is not None:
        m1 = torch.from_numpy(np.ascontiguousarray(p.maps[..., :1])).to(torch.complex64).to(dev)
        x = torch.from_numpy(p.x_true).to(torch.complex64).to(dev)
        got = ctx.normal_apply(m1, x).cpu().numpy().astype(np.complex128)
        out["normal_apply_one_coil_rel_l2"] = float(np.linalg.norm(got - cpu_ref) /
                                                    np.linalg.norm(cpu_ref))
    # split-BF16 MFMA coil mixing against an FP64 matmul, on a 12 x 32 mix of
    # the full-size maps
    rng = np.random.default_rng(7)
    M = rng.standard_normal((Ch, p.n_coils)) + 1j * rng.standard_normal((Ch, p.n_coils))
    maps = torch.from_numpy(np.ascontiguousarray(p.maps)).to(torch.complex64).to(dev)
    got = ctx.coil_mix(maps, M).cpu().numpy().astype(np.complex128)
    ref = p.maps.astype(np.complex64).astype(np.complex128) @ M.T
    out["coil_mix_split_bf16_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    log(f"precision vs FP64: {out}")
    return out


HEADLINE_MAX_CHARS = 4000
# kernel kind (library timer) -> the source file that holds it; a counter
# summary in profiles/ is used for `roofline.traffic` only while the hash of
# that file and of the internal header still match the ones it was taken with
KIND_SOURCES = {"fft_pass": "fft_pass.hip", "interp": "grid.hip", "spread": "grid.hip",
                "grid_normal": "grid.hip", "spread_merge": "grid.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_cones3d.md")


def kernel_source_hash(kind):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2305_06482_amd", "csrc")
    h = hashlib.sha256()
    for f in (KIND_SOURCES.get(kind, ""), "cs_internal.h"):
        path = os.path.join(csrc, f)
        if not f or not os.path.exists(path):
            return None
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, path=TRAFFIC_FILE):
    """HBM bytes per launch of kernel kind from the committed counter summary
    (lines `traffic <kind> <bytes per launch> <source hash>`), or None when
    there is none or the kernel's source changed since it was taken."""
    if not os.path.exists(path):
        return None
    want = kernel_source_hash(kind)
    with open(path) as fh:
        for line in fh:
            f = line.strip().strip("`").split()
            if len(f) == 4 and f[0] == "traffic" and f[1] == kind and f[3] == want:
                return float(f[2])
    return None


def headline(out):
    """The one-line JSON record: the headline metric, the dominant kernel's
    roofline, the CPU baseline and the precision against FP64; the rest of
    the run goes to the detail file."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
            "pct_hbm_roofline", "normal_apply_ms", "min_GBs", "hbm_copy_GBs", "roofline",
            "kernel_frac", "cpu_baseline", "precision", "time_to_1e-3", "detail_file")
    h = {k: out[k] for k in keys if k in out}
    s = json.dumps(h, separators=(",", ":"))
    if len(s) > HEADLINE_MAX_CHARS:
        raise ValueError(f"headline line is {len(s)} characters")
    return s


def kernel_table(prof, geom, Ch, n_sk, n_full, C):
    """Per kernel kind: total ms, launches, and the algorithmic bytes of its
    launches in the profiled steps (sketched applies with Ch coils, full
    applies in chunks of 16)."""
    kb_sk = kernel_bytes(geom, Ch)
    chunks = [16] * (C // 16) + ([C % 16] if C % 16 else [])
    kern = {}
    for name, (ms, cnt) in prof.items():
        entry = {"ms": ms, "launches": cnt}
        if name in kb_sk and cnt:
            per = KERNEL_LAUNCHES_PER_APPLY.get(name, 1)
            tot = kb_sk[name] * per * n_sk
            tot += sum(kernel_bytes(geom, cb)[name] * per for cb in chunks) * n_full
            entry["algorithmic_GB"] = tot / 1e9
            entry["GB/s"] = tot / (ms * 1e-3) / 1e9
            entry["bytes_per_launch"] = tot / cnt
        kern[name] = entry
    return kern


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--K", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="extra steps run with per-kernel HIP events for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="48^3 instance (quick check)")
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file for the full record and the secondary studies")
    ap.add_argument("--studies", action="store_true",
                    help="also run the secondary studies (time to accuracy, batched slices, "
                         "l1-TV, sketch designs, g-factor) into the detail file")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-accuracy runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-slice batch")
    ap.add_argument("--no-tv", action="store_true",
                    help="skip the l1-TV time-to-accuracy runs (48^3 cones)")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the sketching-matrix design ablation (2D radial)")
    ap.add_argument("--no-gfactor", action="store_true",
                    help="skip the Monte-Carlo inverse g-factor of l2 reconstructions")
    ap.add_argument("--tta-ref-iters", type=int, default=2000)
    ap.add_argument("--tta-chunk", type=int, default=100)
    ap.add_argument("--tta-full-iters", type=int, default=3000)
    ap.add_argument("--tta-outer-iters", type=int, default=200)
    ap.add_argument("--no-cart-tta", action="store_true",
                    help="skip the Cartesian time-to-accuracy runs")
    ap.add_argument("--tta-sketch-seeds", type=int, default=3,
                    help="sketch seeds per Algorithm 1 run of the cones time to accuracy")
    # the paper's weight for the cones l1-wavelet reconstruction; at the
    # workload's default 5e-4 plain FISTA is still far from its minimizer
    # after thousands of iterations, which leaves x_inf undefined at 5%
    ap.add_argument("--tta-lam", type=float, default=0.02)
    ap.add_argument("--tta-cart-seeds", type=int, default=5,
                    help="draws of the 320x320 Cartesian problem for the time-to-accuracy "
                         "spread")
    ap.add_argument("--no-cones-tta", action="store_true",
                    help="time to accuracy on the Cartesian problems only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design shards coils with one image all-reduce per apply, "
              "but it is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2305_06482_amd import Context

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    p = synth.make_cones_small() if args.small else synth.make_cones()
    C, V, S = p.n_coils, p.V, p.S
    Ch = V + S
    log(f"inputs generated in {time.time() - t0:.1f} s: shape {p.shape}, "
        f"{p.coords.shape[0]} samples, C={C}, V={V}, S={S}")

    def dt(a, dtype):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(dev)

    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = Context(p.shape, C, "noncart", nsamp=p.coords.shape[0], sigma=1.25, wav_levels=4)
    maps = dt(p.maps, torch.complex64)
    coords = dt(p.coords, torch.float32)
    dcf = dt(p.dcf, torch.float32)
    t0 = time.time()
    ctx.set_operator(maps, coords=coords, dcf=dcf)
    setup_s = time.time() - t0
    log(f"operator set (trajectory sorted and binned) in {setup_s:.2f} s")
    torch.cuda.synchronize()
    # device memory held by the context and its inputs (the library allocates
    # with hipMalloc, outside torch's pool): every coil stays resident
    mem = {"context_and_inputs_bytes": int(free0 - torch.cuda.mem_get_info()[0]),
           "maps_bytes": int(maps.numel() * 8), "total_bytes": int(torch.cuda.mem_get_info()[1])}
    x_true = dt(p.x_true, torch.complex64)
    y = ctx.sense_apply(maps, x_true)
    y += dt(p.noise, torch.complex64) * torch.sqrt(dcf)[:, None].to(torch.complex64)
    del p.noise
    torch.cuda.synchronize()
    mz, my, mx = ctx.grid_shape()
    nz, ny, nx = p.shape
    geom = (nz, ny, nx, mz, my, mx, p.coords.shape[0])

    # untimed preparation: b = A^H y, PCA basis, step size from the first
    # subproblem's power iteration
    t0 = time.time()
    prep = ctx.recon_run(y, mode="sketch", lam=p.lam, T=0, K=args.K, V=V, S=S, seed=p.seed,
                         n_pow=30)
    alpha = prep.alpha
    log(f"prep (b, PCA, power iteration) {time.time() - t0:.1f} s, alpha={alpha:.4g}")

    x = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
    t_idx = 1

    def step():
        nonlocal t_idx
        r = ctx.recon_run(y, mode="sketch", lam=p.lam, T=1, K=args.K, V=V, S=S, seed=p.seed,
                          t0=t_idx, step=alpha, reuse_b=True, x=x)
        t_idx += 1
        return r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # timed region: per-kernel events off; the phase events of recon_run
    # (a few per outer iteration) give the applies' GPU time
    ctx.profile_enable(False)
    results = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    # profiled pass: the same steps with a HIP event pair around every kernel
    # launch on the context stream (the roofline's per-launch durations)
    ctx.profile_enable(True)
    ctx.profile_read()
    presults = [step() for _ in range(max(1, args.profile_steps))]
    prof = ctx.profile_read()
    ctx.profile_enable(False)

    n_sk = sum(r.n_sketch_applies for r in results)
    n_full = sum(r.n_full_applies for r in results)
    ms_sk = sum(r.ms_sketch_normal for r in results)
    ms_full = sum(r.ms_full_normal for r in results)
    b_sk = model_bytes_normal(geom, Ch)
    b_full = model_bytes_normal(geom, C)
    D3 = nz * ny * nx
    bmin_sk = min_bytes_normal(D3, geom[6], 3, Ch)
    bmin_full = min_bytes_normal(D3, geom[6], 3, C)
    gbs = b_sk * n_sk / (ms_sk * 1e-3) / 1e9
    gbs_full = b_full * n_full / (ms_full * 1e-3) / 1e9

    kern = kernel_table(prof, geom, Ch, sum(r.n_sketch_applies for r in presults),
                        sum(r.n_full_applies for r in presults), C)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    roof = None
    if "GB/s" in kern[dom]:
        ach = kern[dom]["GB/s"]
        tr = None if args.small else measured_traffic(dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": tr,
                "avg_launch_ms": round(kern[dom]["ms"] / kern[dom]["launches"], 4),
                "bytes_per_launch": round(kern[dom]["bytes_per_launch"])}

    out = {
        "metric": METRIC,
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("cones3d_48x48x48" if args.small else "cones3d_192x192x128")
                   + f"_N{geom[6]}_C{C}_sketch{V}+{S}_K{args.K}",
                   "grid": [mz, my, mx]},
        "pct_hbm_roofline": round(100 * gbs / HBM_PEAK_GBS, 2),
        "normal_apply_ms": {"sketched": round(ms_sk / max(1, n_sk), 3),
                            "full": round(ms_full / max(1, n_full), 3)},
        "full_normal_GBs": round(gbs_full, 1),
        "phase_ms_per_step": {"full_normal": sum(r.ms_full_normal for r in results) / args.steps,
                              "sketched_normal": ms_sk / args.steps,
                              "prox": sum(r.ms_prox for r in results) / args.steps,
                              "sketch": sum(r.ms_sketch for r in results) / args.steps},
        "model_bytes": {"sketched": b_sk, "full": b_full},
        "min_bytes": {"sketched": bmin_sk, "full": bmin_full},
        "min_GBs": {"sketched": round(bmin_sk * n_sk / (ms_sk * 1e-3) / 1e9, 1),
                    "full": round(bmin_full * n_full / (ms_full * 1e-3) / 1e9, 1)},
        "operator_setup_s": round(setup_s, 3),
        "device_memory": mem,
        "kernels": kern,
        "roofline": roof,
        # every modelled kernel kind's algorithmic bytes per second over the
        # HBM peak, so the kinds beside the dominant one are on record too
        "kernel_frac": {k: round(v["GB/s"] / HBM_PEAK_GBS, 4) for k, v in kern.items()
                        if "GB/s" in v},
        "detail_file": args.detail,
    }
    out["hbm_copy"] = hbm_copy_bandwidth()
    out["hbm_copy_GBs"] = round(out["hbm_copy"]["GB/s"], 1)
    log(f"plain device copy: {out['hbm_copy']['GB/s']:.0f} GB/s")
    cpu_ref = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        out["cpu_baseline"], cpu_ref = cpu_baseline(p, Ch, geom)
        log(f"cpu baseline: {out['cpu_baseline']}")
    out["precision"] = precision_report(ctx, p, Ch, cpu_ref, log)
    if args.studies:
        run_studies(out, args, ctx, y, p, Ch, log)
    os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
    with open(args.detail, "w") as fh:
        json.dump(out, fh, indent=1)
    log(f"full record written to {args.detail}")
    ctx.close()
    print(headline(out), flush=True)


def run_studies(out, args, ctx, y, p, Ch, log):
    """Secondary studies (time to accuracy, batched slices, l1-TV, sketch
    designs, g-factor): written to the detail file only."""
    import synth
    V, S = p.V, p.S
    if not args.no_batched and not args.small:
        out["batched_radial"] = batched_bench(args, log)
    if not args.no_tv and not args.small:
        out["tv_time_to_accuracy"] = tv_tta(args, log)
    if not args.no_ablation and not args.small:
        out["sketch_design_ablation"] = design_ablation(args, log)
    if not args.no_gfactor and not args.small:
        # lam = 1e-2: every design converges and keeps the full-coil
        # g-factor; lam = 1e-3: the R = 3 system is ill conditioned and
        # small-C^ designs stop converging
        out["l2_inverse_gfactor"] = {
            f"lam{lam:g}": gfactor_bench(args, log, lam=lam, designs=((3, 1), (2, 2), (6, 1)))
            for lam in (1e-2, 1e-3)}
    if not args.no_tta:
        log("time-to-accuracy runs")
        tta = {"thresholds": list(TTA_THRESHOLDS)}
        if not args.no_cones_tta:
            net, tinfo = train_warm_start(args, log, lam=args.tta_lam)
            tta["warm_start_training"] = tinfo
            xr = reference_minimizer(ctx, y, p, args.tta_lam, log)
            tta[p.name] = time_to_accuracy(ctx, y, p, args, log, args.tta_ref_iters,
                                           args.tta_full_iters,
                                           [("sketched", 20, 80, "sketch"),
                                            # the design the paper's sketching
                                            # experiments favour: V = C^ - 1, S = 1,
                                            # with longer subproblem solves
                                            ("sketched", 50, 40, "sketch", Ch - 1, 1),
                                            ("sketched", 100, 25, "sketch", Ch - 1, 1),
                                            ("sketched_learned", 100, 25, "learned", Ch - 1, 1)],
                                           args.tta_chunk, cnn=net, lam=args.tta_lam,
                                           x_ref=xr, sketch_seeds=args.tta_sketch_seeds)
            net.close()
        if not args.small and not args.no_cart_tta:
            for pc in (synth.make_cart_small(), synth.make_cart_clinical()):
                tta[pc.name] = cartesian_tta(pc, args, log)
            if args.tta_cart_seeds > 1:
                tta["cart320_seeds"] = cartesian_tta_seeds(tta["cart320"], args, log,
                                                           args.tta_cart_seeds)
        out["time_to_accuracy"] = tta


if __name__ == "__main__":
    main()
