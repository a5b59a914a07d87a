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


def kernel_bytes(geom, cb):
    """Algorithmic bytes per launch of the main kernels for a coil chunk cb."""
    nz, ny, nx, mz, my, mx, N = geom
    D, M = nz * ny * nx, mz * my * mx
    passes = 8 * (cb * (2 * D + 4 * mz * ny * nx + 4 * mz * my * nx + 2 * M) + 2 * D)
    interp = 8 * M * cb + 16 * N + 8 * N * cb
    spread = 8 * N * cb + 16 * N + 8 * M * cb
    return {"fft_pass": passes / 6.0, "interp": interp, "spread": spread}


def cpu_baseline(p, Ch, geom):
    """The FP64 oracle's normal apply for one coil at full size, scaled to the
    Ch coils of a sketched apply."""
    import numpy as np
    from oracle import nufft
    coords = p.coords.astype(np.float32).astype(np.float64)
    dcf = p.dcf.astype(np.float32).astype(np.float64)
    plan = nufft.Plan(p.shape, coords, dcf)
    m1 = p.maps[..., :1]
    x = p.x_true
    t0 = time.perf_counter()
    plan.normal(x, m1)
    dt = time.perf_counter() - t0
    per_apply = dt * Ch
    gbs = model_bytes_normal(geom, Ch) / per_apply / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": (f"one coil of the sketched normal apply at full size "
                       f"({p.shape[0]}x{p.shape[1]}x{p.shape[2]}, {coords.shape[0]} samples), "
                       f"{dt:.1f} s, scaled x{Ch}; NumPy FFT and bincount are single-threaded"),
            "seconds_per_apply": per_apply}


def first_below(dist, thr):
    for i, d in enumerate(dist):
        if d <= thr:
            return i
    return None


def time_to_accuracy(ctx, y, p, args, log):
    """Time to d(x^t) = ||x^t - x_inf|| / ||x_inf|| <= thr (Sec. 3.3.1) for the
    plain full-coil FISTA and for Algorithm 1, both in FP32 on this GPU.

    x_inf is the full-coil problem's minimizer, found by plain FISTA run in
    chunks (momentum restarted per chunk) until one chunk changes x by less
    than 1e-5 relative.  Times are GPU event times on the context stream:
    `loop_ms` covers the iterations up to the first one within thr, `prep_ms`
    the set-up (b = A^H y, step size by power iteration, PCA basis and first
    sketch)."""
    import torch
    thr = args.tta_thr
    C, V, S = p.n_coils, p.V, p.S
    dev = y.device
    t0 = time.time()
    pf = ctx.recon_run(y, mode="full", lam=p.lam, T=0, step=0.0, n_pow=30)
    alpha_f = pf.alpha
    x_inf = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
    change, its = None, 0
    while its < args.tta_ref_iters:
        prev = x_inf.clone()
        ctx.recon_run(y, mode="full", lam=p.lam, T=args.tta_chunk, step=alpha_f,
                      reuse_b=True, x=x_inf)
        its += args.tta_chunk
        change = (torch.linalg.vector_norm(x_inf - prev) /
                  torch.linalg.vector_norm(x_inf)).item()
        log(f"x_inf: {its} full FISTA iterations, last-chunk change {change:.3e}")
        if change < 1e-5:
            break
    ref = {"iterations": its, "chunk": args.tta_chunk, "last_chunk_rel_change": change,
           "wall_s": round(time.time() - t0, 1)}

    def summarize(r, n_full_per_it, n_sk_per_it, pre_full, pre_sk):
        i = first_below(r.dist, thr)
        out = {"prep_ms": r.prep_ms, "iterations_run": len(r.dist),
               "final_dist": r.dist[-1] if r.dist else None, "alpha": r.alpha}
        if i is None:
            out.update({"converged": False})
            return out
        out.update({
            "converged": True, "iterations": i + 1,
            "loop_ms": r.time_ms[i], "total_ms": r.time_ms[i] + r.prep_ms,
            "full_applies": pre_full + (i + 1) * n_full_per_it,
            "sketched_applies": pre_sk + (i + 1) * n_sk_per_it,
        })
        out["coil_ffts"] = 2 * (out["full_applies"] * C + out["sketched_applies"] * (V + S))
        return out

    x = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
    rf = ctx.recon_run(y, mode="full", lam=p.lam, T=args.tta_full_iters, step=0.0, n_pow=30,
                       reuse_b=False, x=x, x_ref=x_inf)
    full = summarize(rf, 1, 0, 31, 0)
    log(f"full-coil FISTA: {full}")

    # PCA basis recomputed so that its cost is part of the sketched set-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    ctx.sketch_build(y, V, S, p.seed, 1, refresh=True, host_outputs=False)
    ev[1].record()
    torch.cuda.synchronize()
    pca_ms = ev[0].elapsed_time(ev[1])
    x = torch.zeros(p.shape, dtype=torch.complex64, device=dev)
    rs = ctx.recon_run(y, mode="sketch", lam=p.lam, T=args.tta_outer_iters, K=args.K, V=V,
                       S=S, seed=p.seed, t0=1, step=0.0, n_pow=30, reuse_b=False, x=x,
                       x_ref=x_inf)
    sk = summarize(rs, 1, args.K, 0, 31)
    sk["pca_ms"] = pca_ms
    if sk.get("converged"):
        sk["total_ms"] += pca_ms
    log(f"sketched (Alg. 1, K={args.K}): {sk}")
    res = {"threshold": thr, "x_inf": ref, "full_coil": full, "sketched": sk,
           "sketched_learned": None}
    if full.get("converged") and sk.get("converged"):
        res["speedup_total"] = full["total_ms"] / sk["total_ms"]
        res["speedup_loop"] = full["loop_ms"] / sk["loop_ms"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--K", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="48^3 instance (quick check)")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-accuracy runs")
    ap.add_argument("--tta-thr", type=float, default=1e-3)
    ap.add_argument("--tta-ref-iters", type=int, default=600)
    ap.add_argument("--tta-chunk", type=int, default=100)
    ap.add_argument("--tta-full-iters", type=int, default=400)
    ap.add_argument("--tta-outer-iters", type=int, default=100)
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

    ctx = Context(p.shape, C, "noncart", nsamp=p.coords.shape[0], sigma=1.25, wav_levels=4)
    maps = dt(p.maps, torch.complex64)
    coords = dt(p.coords, torch.float32)
    dcf = dt(p.dcf, torch.float32)
    t0 = time.time()
    ctx.set_operator(maps, coords=coords, dcf=dcf)
    log(f"operator set (trajectory sorted and binned) in {time.time() - t0:.1f} s")
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
    for _ in range(args.warmup):
        ctx.recon_run(y, mode="sketch", lam=p.lam, T=1, K=args.K, V=V, S=S, seed=p.seed,
                      t0=t_idx, step=alpha, reuse_b=True, x=x)
        t_idx += 1
    torch.cuda.synchronize()
    log("warmup done")

    ctx.profile_enable(True)
    ctx.profile_read()
    results = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        r = ctx.recon_run(y, mode="sketch", lam=p.lam, T=1, K=args.K, V=V, S=S, seed=p.seed,
                          t0=t_idx, step=alpha, reuse_b=True, x=x)
        results.append(r)
        t_idx += 1
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    n_sk = sum(r.n_sketch_applies for r in results)
    n_full = sum(r.n_full_applies for r in results)
    ms_sk = sum(r.ms_sketch_normal for r in results)
    ms_full = sum(r.ms_full_normal for r in results)
    ms_prox = sum(r.ms_prox for r in results)
    ms_sketch = sum(r.ms_sketch for r in results)
    b_sk = model_bytes_normal(geom, Ch)
    b_full = model_bytes_normal(geom, C)
    gbs = b_sk * n_sk / (ms_sk * 1e-3) / 1e9
    gbs_full = b_full * n_full / (ms_full * 1e-3) / 1e9

    # dominant kernel and its roofline
    kb_sk = kernel_bytes(geom, Ch)
    kb_full = kernel_bytes(geom, 16)
    kern = {}
    # the gridding step is the spread kernel plus the merge of its partial
    # tiles: its algorithmic bytes are charged to the pair
    merge_ms = prof.get("spread_merge", (0.0, 0))[0]
    for name, (ms, cnt) in prof.items():
        if name == "spread":
            ms = ms + merge_ms
        entry = {"ms": ms, "launches": cnt}
        if name in kb_sk and cnt:
            per_sk = 6 if name == "fft_pass" else 1
            tot = (kb_sk[name] * per_sk * n_sk + kb_full[name] * per_sk * 2 * n_full)
            entry["algorithmic_GB"] = tot / 1e9
            entry["GB/s"] = tot / (ms * 1e-3) / 1e9
            entry["bytes_per_launch"] = tot / cnt
        kern[name] = entry
    dom = max(kern, key=lambda k: kern[k]["ms"])
    roof = None
    if "GB/s" in kern[dom]:
        ach = kern[dom]["GB/s"]
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "avg_launch_ms": kern[dom]["ms"] / kern[dom]["launches"],
                "bytes_per_launch": kern[dom]["bytes_per_launch"], "traffic": None}

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
                   "grid": [mz, my, mx], "samples_per_coil": geom[6], "coils": C,
                   "sketched_coils": Ch},
        "pct_hbm_roofline": round(100 * gbs / HBM_PEAK_GBS, 2),
        "normal_apply_ms": {"sketched": ms_sk / max(1, n_sk), "full": ms_full / max(1, n_full)},
        "full_normal_GBs": round(gbs_full, 1),
        "phase_ms_per_step": {"full_normal": ms_full / args.steps,
                              "sketched_normal": ms_sk / args.steps,
                              "prox": ms_prox / args.steps, "sketch": ms_sketch / args.steps},
        "model_bytes": {"sketched": b_sk, "full": b_full},
        "kernels": kern,
        "roofline": roof,
    }
    if not args.no_tta:
        log("time-to-accuracy runs")
        out["time_to_accuracy"] = time_to_accuracy(ctx, y, p, args, log)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(p, Ch, geom)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
