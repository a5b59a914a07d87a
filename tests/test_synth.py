"""Synthetic input generators: determinism and the stated workload shapes."""
import numpy as np

import synth


def test_phantom_deterministic_and_normalised():
    a = synth.phantom((32, 32), 7)
    b = synth.phantom((32, 32), 7)
    c = synth.phantom((32, 32), 8)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert abs(np.abs(a).max() - 1.0) < 1e-12
    v = synth.phantom((8, 12, 16), 3)
    assert v.shape == (8, 12, 16) and abs(np.abs(v).max() - 1.0) < 1e-12


def test_maps_unit_rss():
    for shape, C in [((24, 20), 8), ((6, 10, 12), 12)]:
        m = synth.coil_maps(shape, C, 1)
        assert m.shape == shape + (C,)
        rss = np.sqrt(np.sum(np.abs(m) ** 2, axis=-1))
        assert np.allclose(rss, 1.0, atol=1e-12)


def test_mask_1d_vd_rate_and_centre():
    m = synth.mask_1d_vd(128, 128, 1003)
    assert m.shape == (128, 128)
    lines = m[:, 0].astype(bool)
    assert lines.sum() == 32                                  # R = 4
    assert np.all(m == m[:, :1])                              # kx fully sampled
    centred = np.fft.fftshift(lines)
    assert centred[64 - 12:64 + 12].all()                     # 24 centre lines


def test_mask_poisson_rate():
    m = synth.mask_poisson(64, 64, 5, accel=4.0, calib=8)
    target = 64 * 64 / 4.0
    assert abs(m.sum() - target) <= 0.01 * target + 1
    c = np.fft.fftshift(m)
    assert c[32 - 4:32 + 4, 32 - 4:32 + 4].all()


def test_trajectories_in_bounds():
    k = synth.radial_traj(64, 10)
    assert k.shape == (10 * 128, 2)
    assert k.min() >= -32 and k.max() < 32
    w = synth.radial_dcf(k, 64)
    assert np.all(w > 0)
    kc = synth.cones_traj((16, 24, 24), 200, 32, seed=1)
    assert kc.shape == (200 * 32, 3)
    lim = np.array([12, 12, 8])
    assert np.all(kc >= -lim) and np.all(kc < lim)
    wc = synth.cones_dcf(kc, (16, 24, 24))
    assert np.all(wc > 0)


def test_noise_statistics():
    n = synth.complex_noise((200000,), 2.0, 9)
    assert abs(np.mean(np.abs(n) ** 2) - 4.0) < 0.05
    assert abs(np.var(n.real) - 2.0) < 0.05


def test_batched_specs():
    specs = synth.batched_radial_specs(64)
    assert len(specs) == 64
    for s in specs:
        assert s["n"] in (128, 192, 256, 384)
        assert 64 <= s["spokes"] <= 402
        assert 8 <= s["coils"] <= 32
        assert 2 <= s["V"] <= min(8, (s["coils"] - 1) // 2)
        assert s["V"] + s["S"] < s["coils"]
