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
