"""Seeded synthetic inputs shaped like the paper's workloads (Section 3.1).

The paper's knee, radial-liver and 3D-cones acquisitions are not available, so
every input here is generated: an ellipse/ellipsoid phantom, smooth
Gaussian-profile coil sensitivities, Cartesian sampling masks, radial and
cones-like non-Cartesian trajectories with their density compensation, and
complex Gaussian noise.

This module holds none of the reconstruction arithmetic (no Fourier
transform, no sensitivity multiply, no sketching): it only draws inputs.  Both
the CPU oracle and the GPU path consume what it returns.  Random streams use
``numpy.random.Generator(PCG64(seed))`` so that every array is reproducible.

Layout conventions (shared by the oracle and the GPU library):
  * image / maps pixel index is row-major ``[nz][ny][nx]`` (2D: ``[ny][nx]``),
    centred coordinate of index ``i`` along an axis of length ``n`` is
    ``i - n // 2``;
  * coil sensitivities are pixel-major with the coil index fastest:
    ``maps[..., c]``;
  * Cartesian masks are stored in the non-centred FFT layout (DC at index 0);
  * non-Cartesian coordinates are ``[N, ndim]`` in cycles/FOV, column 0 = x
    (fastest image axis), column 1 = y, column 2 = z, each within
    ``[-n_a/2, n_a/2)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

# Stream identifiers for seeding: seed = 1000 * config + stream.
STREAM_PHANTOM = 1
STREAM_MAPS = 2
STREAM_SAMPLING = 3
STREAM_NOISE = 4
STREAM_SKETCH = 5

GOLDEN_ANGLE_DEG = 111.246117975  # 180 * (sqrt(5) - 1) / 2 ... radial increment
GOLDEN_RATIO = (1.0 + math.sqrt(5.0)) / 2.0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _axis_coords(n: int) -> np.ndarray:
    """Normalised FOV coordinate in [-1, 1) of each index along an axis."""
    return (np.arange(n) - n // 2) / (n / 2.0)


def _grid(shape):
    """Normalised coordinates, returned in (x, y[, z]) order, each broadcast to
    the image shape (row-major, slowest axis first in ``shape``)."""
    axes = [_axis_coords(n) for n in shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    return mesh[::-1]  # x first


def _random_rotation(g: np.random.Generator, ndim: int) -> np.ndarray:
    if ndim == 2:
        a = g.uniform(0.0, math.pi)
        return np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    q, r = np.linalg.qr(g.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def phantom(shape, seed: int, n_ellipses: int = 10) -> np.ndarray:
    """Random-ellipse (2D) or random-ellipsoid (3D) complex phantom.

    Centres U[-0.5, 0.5], semi-axes U[0.05, 0.4], uniform random rotation,
    amplitude U[0.2, 1] times exp(i*phi) with phi ~ U[-pi, pi).  The ellipses
    are summed and the result is scaled to max |x| = 1.
    """
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    g = rng(seed)
    coords = _grid(shape)  # x, y[, z]
    pts = np.stack([c.ravel() for c in coords], axis=1)  # [D, ndim]
    img = np.zeros(pts.shape[0], dtype=np.complex128)
    for _ in range(n_ellipses):
        centre = g.uniform(-0.5, 0.5, size=ndim)
        semi = g.uniform(0.05, 0.4, size=ndim)
        rot = _random_rotation(g, ndim)
        amp = g.uniform(0.2, 1.0) * np.exp(1j * g.uniform(-math.pi, math.pi))
        local = (pts - centre) @ rot  # coordinates in the ellipse frame
        inside = np.sum((local / semi) ** 2, axis=1) <= 1.0
        img[inside] += amp
    img = img.reshape(shape)
    m = np.abs(img).max()
    if m > 0:
        img /= m
    return img


def coil_maps(shape, n_coils: int, seed: int, width: float = 0.8,
              radius: float = 1.5) -> np.ndarray:
    """Smooth Gaussian-profile sensitivities, normalised to unit root-sum-of-squares.

    2D: coil centres on a circle of radius 1.5 at angles 2*pi*c/C.
    3D: two rings of C/2 coils (radius 1.5 in x-y) at z = +0.6 and z = -0.6.
    Each coil gets a random constant phase.  Returned layout ``shape + (C,)``.
    """
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    g = rng(seed)
    coords = _grid(shape)
    centres = []
    if ndim == 2:
        for c in range(n_coils):
            a = 2 * math.pi * c / n_coils
            centres.append((radius * math.cos(a), radius * math.sin(a)))
    else:
        half = (n_coils + 1) // 2
        for c in range(n_coils):
            ring = 0 if c < half else 1
            k = c if ring == 0 else c - half
            nring = half if ring == 0 else n_coils - half
            a = 2 * math.pi * k / nring + (0.0 if ring == 0 else math.pi / nring)
            centres.append((radius * math.cos(a), radius * math.sin(a),
                            0.6 if ring == 0 else -0.6))
    phases = g.uniform(-math.pi, math.pi, size=n_coils)
    maps = np.empty(shape + (n_coils,), dtype=np.complex128)
    for c in range(n_coils):
        d2 = sum((coords[a] - centres[c][a]) ** 2 for a in range(ndim))
        maps[..., c] = np.exp(-d2 / (2 * width ** 2)) * np.exp(1j * phases[c])
    rss = np.sqrt(np.sum(np.abs(maps) ** 2, axis=-1, keepdims=True))
    return maps / rss


def mask_1d_vd(ny: int, nx: int, seed: int, n_center: int = 24,
               accel: int = 4) -> np.ndarray:
    """1D variable-density random mask over ky lines (kx fully sampled).

    The ``n_center`` central lines are always sampled; the remaining
    ``ny/accel - n_center`` lines are drawn without replacement with
    probability proportional to (1 - 2|ky|/ny)^3.  Returned as uint8
    ``[ny][nx]`` in the non-centred layout.
    """
    g = rng(seed)
    ky = np.arange(ny) - ny // 2
    lines = np.zeros(ny, dtype=bool)
    centre = np.abs(ky + 0.5) < n_center / 2.0
    lines[centre] = True
    n_total = ny // accel
    n_extra = n_total - int(lines.sum())
    cand = np.flatnonzero(~lines)
    p = (1.0 - 2.0 * np.abs(ky[cand]) / ny) ** 3
    p = p / p.sum()
    pick = g.choice(cand, size=n_extra, replace=False, p=p)
    lines[pick] = True
    m = np.repeat(lines[:, None], nx, axis=1)
    return np.fft.ifftshift(m).astype(np.uint8)


def _poisson_disc(ny: int, nx: int, scale: float, g_seed: int) -> np.ndarray:
    """Variable-density Poisson-disc sampling by random sequential acceptance.

    Grid points are visited in a seeded random order; a candidate at centred
    k is accepted when no accepted point lies closer than
    r(k) = scale * (1 + 2 |k| / k_max).
    """
    g = rng(g_seed)
    ky = (np.arange(ny) - ny // 2)[:, None]
    kx = (np.arange(nx) - nx // 2)[None, :]
    kmax = math.hypot(ny / 2, nx / 2)
    r = scale * (1.0 + 2.0 * np.sqrt(ky ** 2 + kx ** 2) / kmax)
    order = g.permutation(ny * nx)
    acc = np.zeros((ny, nx), dtype=bool)
    for idx in order:
        y, x = divmod(int(idx), nx)
        rad = r[y, x]
        h = int(math.ceil(rad))
        y0, y1 = max(0, y - h), min(ny, y + h + 1)
        x0, x1 = max(0, x - h), min(nx, x + h + 1)
        win = acc[y0:y1, x0:x1]
        if win.any():
            yy, xx = np.nonzero(win)
            if np.min((yy + y0 - y) ** 2 + (xx + x0 - x) ** 2) < rad * rad:
                continue
        acc[y, x] = True
    return acc


@lru_cache(maxsize=8)
def _mask_poisson_cached(ny, nx, seed, accel, calib):
    target = ny * nx / accel
    lo, hi = 0.3, 6.0
    best = None
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        m = _poisson_disc(ny, nx, mid, seed)
        cy = np.abs(np.arange(ny) - ny // 2 + 0.5) < calib / 2.0
        cx = np.abs(np.arange(nx) - nx // 2 + 0.5) < calib / 2.0
        m[np.ix_(cy, cx)] = True
        cnt = int(m.sum())
        best = m
        if abs(cnt - target) <= 0.01 * target:
            break
        if cnt > target:
            lo = mid
        else:
            hi = mid
    return np.fft.ifftshift(best).astype(np.uint8)


def mask_poisson(ny: int, nx: int, seed: int, accel: float = 6.0,
                 calib: int = 24) -> np.ndarray:
    """2D variable-density Poisson-disc mask with a fully sampled
    ``calib x calib`` centre, radius scale bisected to D/accel +- 1% samples.
    uint8 ``[ny][nx]``, non-centred layout."""
    return _mask_poisson_cached(int(ny), int(nx), int(seed), float(accel),
                                int(calib)).copy()


def mask_regular(ny: int, nx: int, accel: int = 3, n_center: int = 0) -> np.ndarray:
    """Regular undersampling of every ``accel``-th ky line."""
    ky = np.arange(ny) - ny // 2
    lines = (ky % accel) == 0
    if n_center:
        lines |= np.abs(ky + 0.5) < n_center / 2.0
    m = np.repeat(lines[:, None], nx, axis=1)
    return np.fft.ifftshift(m).astype(np.uint8)


def radial_traj(n: int, n_spokes: int, oversamp: int = 2,
                angle_deg: float = GOLDEN_ANGLE_DEG) -> np.ndarray:
    """2D radial spokes with a fixed angular increment.

    Each spoke has ``oversamp * n`` samples at spacing 1/oversamp cycles/FOV,
    k = (j - n*oversamp/2) / oversamp, so every sample lies in [-n/2, n/2).
    Returns ``[n_spokes * oversamp * n, 2]`` (columns x, y).
    """
    ns = oversamp * n
    kr = (np.arange(ns) - ns // 2) / oversamp
    ang = np.deg2rad(angle_deg) * np.arange(n_spokes)
    kx = np.cos(ang)[:, None] * kr[None, :]
    ky = np.sin(ang)[:, None] * kr[None, :]
    k = np.stack([kx.ravel(), ky.ravel()], axis=1)
    return np.clip(k, -n / 2, n / 2 - 1e-6)


def radial_dcf(coords: np.ndarray, n: int) -> np.ndarray:
    """Ramp density compensation max(|k|, 1/4) / (n/2), rescaled so that the
    weights sum to the area of the sampled disc in Nyquist units."""
    kr = np.sqrt(np.sum(coords ** 2, axis=1))
    w = np.maximum(kr, 0.25) / (n / 2.0)
    return w * (math.pi * (n / 2.0) ** 2 / w.sum())


def cones_traj(shape, n_readouts: int, n_samples: int, n_cones: int = 36,
               seed: int = 3, turns: float = 2.0) -> np.ndarray:
    """Cones-like 3D trajectory.

    Cone polar angles are uniform in cos(theta) over ``n_cones`` cones; each
    cone gets a number of readouts proportional to sin(theta) (total
    ``n_readouts``).  Along readout r of a cone, with s = (j + 1/2)/n_samples,
    k(s) = s * (kx_max sin(th) cos(psi), ky_max sin(th) sin(psi), kz_max cos(th)),
    psi(s) = psi0 + 2*pi*turns*s, where psi0 steps by the golden ratio.
    ``shape`` is the image shape (nz, ny, nx); k_a max = n_a / 2.
    Returns ``[n_readouts * n_samples, 3]`` (columns x, y, z).
    """
    nz, ny, nx = (int(s) for s in shape)
    g = rng(seed)
    cos_th = -1.0 + (2.0 * np.arange(n_cones) + 1.0) / n_cones
    th = np.arccos(cos_th)
    wts = np.sin(th)
    counts = np.floor(wts / wts.sum() * n_readouts).astype(int)
    rem = n_readouts - counts.sum()
    frac = wts / wts.sum() * n_readouts - counts
    counts[np.argsort(-frac, kind="stable")[:rem]] += 1
    s = (np.arange(n_samples) + 0.5) / n_samples
    offset = g.uniform(0.0, 1.0)
    out = []
    r_global = 0
    for ci in range(n_cones):
        for _ in range(counts[ci]):
            psi0 = 2 * math.pi * ((offset + r_global / GOLDEN_RATIO) % 1.0)
            psi = psi0 + 2 * math.pi * turns * s
            st, ct = math.sin(th[ci]), math.cos(th[ci])
            kx = s * (nx / 2.0) * st * np.cos(psi)
            ky = s * (ny / 2.0) * st * np.sin(psi)
            kz = s * (nz / 2.0) * ct * np.ones_like(s)
            out.append(np.stack([kx, ky, kz], axis=1))
            r_global += 1
    k = np.concatenate(out, axis=0)
    lim = np.array([nx / 2.0, ny / 2.0, nz / 2.0])
    return np.clip(k, -lim, lim - 1e-6)


def cones_dcf(coords: np.ndarray, shape, s0: float = 0.05) -> np.ndarray:
    """Density compensation w = max(s^2, s0^2) with s the radius normalised by
    the per-axis k_max, rescaled so that the weights sum to the volume of the
    sampled ellipsoid in Nyquist units."""
    nz, ny, nx = shape
    lim = np.array([nx / 2.0, ny / 2.0, nz / 2.0])
    s = np.sqrt(np.sum((coords / lim) ** 2, axis=1))
    w = np.maximum(s ** 2, s0 ** 2)
    vol = 4.0 / 3.0 * math.pi * lim[0] * lim[1] * lim[2]
    return w * (vol / w.sum())


def complex_noise(shape, sigma: float, seed: int) -> np.ndarray:
    """Circular complex Gaussian CN(0, sigma^2): re, im ~ N(0, sigma^2 / 2)."""
    g = rng(seed)
    s = sigma / math.sqrt(2.0)
    return s * g.standard_normal(shape) + 1j * s * g.standard_normal(shape)


# ---------------------------------------------------------------------------
# Workload configurations (sizes of the paper's Cartesian, radial and cones
# experiments, Section 3.1 and Section 3.3)
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    kind: str                 # "cart" or "noncart"
    shape: tuple              # image shape, slowest axis first
    x_true: np.ndarray        # complex128 image
    maps: np.ndarray          # complex128, shape + (C,)
    mask: np.ndarray | None   # uint8 image-shaped (Cartesian)
    coords: np.ndarray | None  # [N, ndim] float64 (non-Cartesian)
    dcf: np.ndarray | None    # [N] float64 (non-Cartesian)
    noise: np.ndarray         # complex128, [N, C] (Cartesian: [D, C])
    V: int
    S: int
    lam: float
    T: int
    K: int
    seed: int

    @property
    def n_coils(self):
        return self.maps.shape[-1]


def make_cart_small(seed_base: int = 1000) -> Problem:
    """128x128, 8 coils, 1D variable-density mask R=4 with 24 centre lines,
    sketch 2 PCA + 2 Rademacher, lambda 1e-3, 20 outer iterations."""
    shape = (128, 128)
    x = phantom(shape, seed_base + STREAM_PHANTOM)
    maps = coil_maps(shape, 8, seed_base + STREAM_MAPS)
    mask = mask_1d_vd(128, 128, seed_base + STREAM_SAMPLING)
    noise = complex_noise((128 * 128, 8), 1e-3, seed_base + STREAM_NOISE)
    return Problem("cart128", "cart", shape, x, maps, mask, None, None, noise,
                   V=2, S=2, lam=1e-3, T=20, K=5, seed=seed_base + STREAM_SKETCH)


def make_cart_clinical(seed_base: int = 2000) -> Problem:
    """320x320, 32 coils, 2D Poisson-disc mask R=6 with a 24x24 calibration
    region, sketch 4 PCA + 4 Rademacher, lambda 1e-3, 30 outer iterations."""
    shape = (320, 320)
    x = phantom(shape, seed_base + STREAM_PHANTOM)
    maps = coil_maps(shape, 32, seed_base + STREAM_MAPS)
    mask = mask_poisson(320, 320, seed_base + STREAM_SAMPLING)
    noise = complex_noise((320 * 320, 32), 1e-3, seed_base + STREAM_NOISE)
    return Problem("cart320", "cart", shape, x, maps, mask, None, None, noise,
                   V=4, S=4, lam=1e-3, T=30, K=5, seed=seed_base + STREAM_SKETCH)


def make_cones(shape=(128, 192, 192), n_readouts=18000, n_samples=512,
               n_coils=32, V=6, S=6, seed_base: int = 3000,
               lam: float = 5e-4, T: int = 30, K: int = 5) -> Problem:
    """3D cones-like workload: 192x192x128 volume, 18000 readouts x 512
    samples, 32 coils, sketch 6 PCA + 6 Rademacher.  Smaller instances use the
    same generators with smaller arguments."""
    shape = tuple(int(s) for s in shape)
    x = phantom(shape, seed_base + STREAM_PHANTOM)
    maps = coil_maps(shape, n_coils, seed_base + STREAM_MAPS)
    coords = cones_traj(shape, n_readouts, n_samples, seed=seed_base + STREAM_SAMPLING)
    dcf = cones_dcf(coords, shape)
    noise = complex_noise((coords.shape[0], n_coils), 1e-3, seed_base + STREAM_NOISE)
    return Problem("cones", "noncart", shape, x, maps, None, coords, dcf, noise,
                   V=V, S=S, lam=lam, T=T, K=K, seed=seed_base + STREAM_SKETCH)


def make_cones_small(seed_base: int = 3000) -> Problem:
    """The 48^3 instance of the cones workload: 1125 readouts x 128 samples."""
    return make_cones(shape=(48, 48, 48), n_readouts=1125, n_samples=128,
                      seed_base=seed_base)


def make_radial(n: int, n_spokes: int, n_coils: int, V: int, S: int,
                seed_base: int = 4000, lam: float = 1e-3, T: int = 20,
                K: int = 5) -> Problem:
    """2D golden-angle radial slice with 2x-oversampled readouts."""
    shape = (n, n)
    x = phantom(shape, seed_base + STREAM_PHANTOM)
    maps = coil_maps(shape, n_coils, seed_base + STREAM_MAPS)
    coords = radial_traj(n, n_spokes)
    dcf = radial_dcf(coords, n)
    noise = complex_noise((coords.shape[0], n_coils), 1e-3, seed_base + STREAM_NOISE)
    return Problem(f"radial{n}", "noncart", shape, x, maps, None, coords, dcf, noise,
                   V=V, S=S, lam=lam, T=T, K=K, seed=seed_base + STREAM_SKETCH)


def batched_radial_specs(n_slices: int = 64, seed: int = 4003):
    """Per-slice sizes of the batched radial workload: matrix in
    {128,192,256,384}, spokes U[64,402], coils U[8,32], V U[2, min(8,(C-1)//2)],
    S = V."""
    g = rng(seed)
    specs = []
    for _ in range(n_slices):
        n = int(g.choice([128, 192, 256, 384]))
        spokes = int(g.integers(64, 403))
        c = int(g.integers(8, 33))
        v = int(g.integers(2, min(8, (c - 1) // 2) + 1))
        specs.append(dict(n=n, spokes=spokes, coils=c, V=v, S=v))
    return specs
