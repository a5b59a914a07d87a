"""The image-quality metrics the benchmark reports (NRMSE, SSIM, HFEN) on
cases with known answers."""
import numpy as np

import bench


def test_identical_images_are_perfect():
    g = np.random.default_rng(0)
    x = g.standard_normal((24, 20)) + 1j * g.standard_normal((24, 20))
    q = bench.image_quality(x, x)
    assert q["nrmse"] == 0.0 and q["hfen"] == 0.0
    assert abs(q["ssim"] - 1.0) < 1e-12


def test_metrics_worsen_with_noise_and_blur():
    import synth
    ref = synth.phantom((48, 48), 3)
    g = np.random.default_rng(1)
    small = bench.image_quality(ref + 0.01 * g.standard_normal(ref.shape), ref)
    large = bench.image_quality(ref + 0.1 * g.standard_normal(ref.shape), ref)
    assert small["ssim"] > large["ssim"] and small["hfen"] < large["hfen"]
    assert small["nrmse"] < large["nrmse"]
    from scipy import ndimage
    blurred = ndimage.gaussian_filter(np.abs(ref), 2.0, mode="wrap")
    q = bench.image_quality(blurred, ref)
    # blurring removes high frequencies: HFEN suffers much more than NRMSE
    assert q["hfen"] > 1.5 * q["nrmse"] and q["ssim"] < 1.0


def test_ssim_of_a_scaled_image():
    # SSIM's luminance/contrast terms: a uniformly scaled copy loses similarity
    import synth
    ref = np.abs(synth.phantom((32, 32), 4))
    assert bench.image_quality(0.5 * ref, ref)["ssim"] < bench.image_quality(0.9 * ref, ref)["ssim"] < 1.0


def test_byte_models_of_the_normal_apply():
    # 3D cones, 192 x 192 x 128, 9.216 M samples, grid 240 x 240 x 160:
    # 1.129 GB compulsory and 9.764 GB modelled for 12 coils, 2.64 GB and
    # 25.67 GB for 32 (the per-stage tally of the workload)
    D, N = 192 * 192 * 128, 9216000
    geom = (128, 192, 192, 160, 240, 240, N)
    assert abs(bench.min_bytes_normal(D, N, 3, 12) / 1e9 - 1.129) < 1e-3
    assert abs(bench.model_bytes_normal(geom, 12) / 1e9 - 9.764) < 1e-3
    assert abs(bench.min_bytes_normal(D, N, 3, 32) / 1e9 - 2.64) < 5e-3
    assert abs(bench.model_bytes_normal(geom, 32) / 1e9 - 25.67) < 5e-3
    # 2D, n = 256 on a 320 x 320 grid, stage by stage per coil: maps read
    # twice; forward pass 1 writes 320 x 256, pass 2 reads it and writes the
    # grid; interpolation reads the grid, spreading writes it; the adjoint
    # passes mirror the forward ones
    n, m, N2, C = 256, 320, 402 * 512, 5
    stages = [2 * n * n, m * n, m * n + m * m, m * m, m * m, m * m + m * n, m * n]
    per_coil = 8 * sum(stages)
    want = C * per_coil + 2 * 8 * n * n + 12 * N2
    assert bench.model_bytes_normal_2d(n, n, m, m, N2, C) == want
    assert bench.min_bytes_normal(n * n, N2, 2, C) == 8 * n * n * (2 + 2 * C) + 12 * N2


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU only" in r.stdout + r.stderr


def _stub_record():
    # a full record as main() builds it, with the bulky fields the headline
    # leaves to the detail file
    return {
        "metric": bench.METRIC, "value": 1234.5, "unit": "GB/s", "n_gpus": 1, "steps": 20,
        "warmup": 5, "ms_per_step": 50.0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cones3d_192x192x128_N9216000_C32_sketch6+6_K5",
                   "grid": [160, 240, 240]},
        "pct_hbm_roofline": 15.4, "normal_apply_ms": {"sketched": 7.9, "full": 20.0},
        "min_GBs": {"sketched": 143.0, "full": 130.0}, "hbm_copy_GBs": 4800.0,
        "roofline": {"bound": "hbm", "kernel": "spread", "achieved": 500.0, "peak": 8000.0,
                     "unit": "GB/s", "frac": 0.0625, "traffic": None, "avg_launch_ms": 2.0,
                     "bytes_per_launch": 1.0e9},
        "kernel_frac": {"fft_pass": 0.38, "interp": 0.13, "spread": 0.1},
        "cpu_baseline": {"value": 0.4, "unit": "GB/s", "cores": 12, "kind": "oracle",
                         "sample": "x" * 200, "seconds_per_apply": 25.0},
        "precision": {"normal_apply_one_coil_rel_l2": 4e-7, "coil_mix_split_bf16_rel_l2": 1e-7},
        "detail_file": "gpurun_out/bench_detail.json",
        "kernels": {f"k{i}": {"ms": 1.0, "launches": 10, "GB/s": 1.0} for i in range(50)},
        "time_to_accuracy": {"runs": ["y" * 1000] * 40},
    }


def test_headline_line_is_compact_and_complete():
    # the driver keeps only the tail of the run's output: the last line must
    # stay small and still carry the metric, the roofline and the baseline
    import json
    rec = _stub_record()
    line = bench.headline(rec)
    assert len(line) < 4096 and "\n" not in line
    h = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline", "precision"):
        assert k in h, k
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in h["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in h["cpu_baseline"], k
    assert "kernels" not in h and "time_to_accuracy" not in h
    assert h["kernel_frac"]["spread"] == 0.1
    assert h["config"]["workload"].startswith("cones3d")


def test_headline_refuses_an_oversized_line():
    rec = _stub_record()
    rec["config"] = {"workload": "w" * 5000}
    import pytest
    with pytest.raises(ValueError):
        bench.headline(rec)


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path):
    # a counter summary names the source hash it was taken with; a changed
    # kernel source (another hash) gives no traffic figure
    h = bench.kernel_source_hash("fft_pass")
    assert h is not None and len(h) == 16
    f = tmp_path / "t.md"
    f.write_text(f"`traffic fft_pass 123456789 {h}`\n`traffic interp 5 0000000000000000`\n")
    assert bench.measured_traffic("fft_pass", str(f)) == 123456789.0
    assert bench.measured_traffic("interp", str(f)) is None
    assert bench.measured_traffic("spread", str(tmp_path / "missing.md")) is None


def test_cpu_baseline_runs_the_oracle_in_parallel_workers():
    # the baseline times one whole sketched apply, one coil per worker, and
    # returns the oracle's first-coil result for the precision report
    from types import SimpleNamespace
    import synth
    from oracle import nufft
    shape = (8, 12, 10)
    g = np.random.default_rng(3)
    N = 300
    coords = np.stack([g.uniform(-n / 2, n / 2, N) for n in shape[::-1]], axis=1)
    dcf = g.uniform(0.5, 1.5, N)
    maps = synth.coil_maps(shape, 3, 4)
    x = synth.phantom(shape, 5)
    p = SimpleNamespace(coords=coords, dcf=dcf, maps=maps, x_true=x, shape=shape)
    geom = shape + nufft.grid_shape(shape, 1.25) + (N,)
    rec, ref = bench.cpu_baseline(p, 3, geom, max_workers=2)
    assert rec["kind"] == "oracle" and rec["cores"] == 2 and rec["value"] > 0
    plan = nufft.Plan(shape, coords.astype(np.float32).astype(np.float64),
                      dcf.astype(np.float32).astype(np.float64))
    want = plan.normal(x.astype(np.complex64).astype(np.complex128),
                       maps[..., :1].astype(np.complex64).astype(np.complex128))
    assert np.allclose(ref, want, rtol=0, atol=1e-12 * np.abs(want).max())
