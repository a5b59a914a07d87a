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
