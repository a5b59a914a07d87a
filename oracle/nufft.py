"""Non-Cartesian multi-coil SENSE operator with a Kaiser-Bessel NUFFT (oracle,
float64; test infrastructure: only tests, the smoke check and the
benchmark's CPU baseline use it).

Sec. 2.1, Eq. 1 defines the forward model as the non-uniform DFT

    k_c[i] = D^{-1/2} sum_d c_c[d] x[d] exp(-i 2 pi f_i . r_d) + n_c[i]

and states that F~_n is implemented as a NUFFT (Beatty et al. 2005); with
density compensation A = W^1/2 F C, y = W^1/2 k (Sec. 2.1.1) and the coil-wise
operator y_c = w^1/2 * NUFFT(c_c * x) (Eq. 5).

Readings (the paper gives no NUFFT details beyond the citation):
  * Eq. 1's garbled exponent is read per axis as exp(-i 2 pi sum_a k_a r_a / n_a)
    with centred image coordinates r_a = i_a - n_a//2 and k in cycles/FOV.
  * Oversampled grid m_a = round(sigma * n_a); a sample sits at grid
    coordinate u_a = k_a * m_a / n_a.
  * Kaiser-Bessel kernel of width W grid cells,
    phi(t) = I0(beta sqrt(1 - (2t/W)^2)) for |t| <= W/2, with Beatty's
    beta = pi sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8).
  * Taps of a sample are g = floor(u) - (W/2 - 1) + j, j = 0..W-1 (for W = 4:
    floor(u)-1 .. floor(u)+2, a half-open window (u - W/2, u + W/2]); grid
    indices are taken modulo m_a.
  * Deapodisation divides by the kernel's continuous Fourier transform
    Phi(nu) = W sinh(sqrt(beta^2 - (pi W nu)^2)) / sqrt(beta^2 - (pi W nu)^2)
    at nu = r_a / m_a.
  * The oversampled DFT is the unnormalised sum over the zero-padded image
    (image index r placed at grid index r mod m); the 1/sqrt(D) of Eq. 1 is
    applied once.

Steps of the forward operator (for each coil): multiply by the map, divide by
the deapodisation, zero-pad, FFT, interpolate with the KB kernel, scale by
1/sqrt(D) and by sqrt(w).  The adjoint is the exact adjoint of each step.

Layout: image ``shape`` = (nz, ny, nx) or (ny, nx); coordinates ``[N, ndim]``
with column 0 = x (last array axis); data ``[N, C]``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import i0


def kb_beta(W: int, sigma: float) -> float:
    """Beatty et al. 2005 choice of the Kaiser-Bessel shape parameter."""
    return math.pi * math.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def kb_kernel(t, W: int, beta: float):
    """phi(t) = I0(beta sqrt(1 - (2t/W)^2)) inside |t| <= W/2, else 0."""
    t = np.asarray(t, dtype=np.float64)
    z = 1.0 - (2.0 * t / W) ** 2
    out = np.where(z >= 0, i0(beta * np.sqrt(np.maximum(z, 0.0))), 0.0)
    return out


def kb_ft(nu, W: int, beta: float):
    """Continuous Fourier transform of ``kb_kernel`` at frequency nu
    (cycles per grid cell)."""
    nu = np.asarray(nu, dtype=np.float64)
    a = beta ** 2 - (math.pi * W * nu) ** 2
    s = np.sqrt(np.abs(a))
    with np.errstate(invalid="ignore", divide="ignore"):
        pos = W * np.sinh(s) / s
        neg = W * np.sin(s) / s
    return np.where(a > 0, pos, np.where(a < 0, neg, W))


def grid_shape(shape, sigma: float):
    return tuple(int(round(sigma * n)) for n in shape)


def deapod(shape, gshape, W: int, beta: float) -> np.ndarray:
    """Separable deapodisation Phi(r_a / m_a) over the image (centred r)."""
    out = np.ones(shape)
    for a, (n, m) in enumerate(zip(shape, gshape)):
        r = np.arange(n) - n // 2
        v = kb_ft(r / m, W, beta)
        sh = [1] * len(shape)
        sh[a] = n
        out = out * v.reshape(sh)
    return out


class Plan:
    """Geometry of one non-Cartesian operator: per-axis taps and weights."""

    def __init__(self, shape, coords, dcf, sigma: float = 1.25, W: int = 4,
                 beta: float | None = None):
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.sigma = sigma
        self.W = W
        self.beta = kb_beta(W, sigma) if beta is None else beta
        self.gshape = grid_shape(self.shape, sigma)
        self.D = int(np.prod(self.shape))
        self.coords = np.asarray(coords, dtype=np.float64)
        self.N = self.coords.shape[0]
        self.dcf = None if dcf is None else np.asarray(dcf, dtype=np.float64)
        # per array axis a (0 = slowest): taps [N, W] (mod m) and weights [N, W]
        self.taps = []
        self.wts = []
        for a in range(self.ndim):
            n, m = self.shape[a], self.gshape[a]
            k = self.coords[:, self.ndim - 1 - a]
            u = k * m / n
            base = np.floor(u).astype(np.int64) - (W // 2 - 1)
            g = base[:, None] + np.arange(W)[None, :]
            self.taps.append(np.mod(g, m))
            self.wts.append(kb_kernel(u[:, None] - g, W, self.beta))
        self.apod = deapod(self.shape, self.gshape, W, self.beta)

    # -- gridding -----------------------------------------------------------
    def _tap_iter(self):
        W = self.W
        for combo in np.ndindex(*([W] * self.ndim)):
            w = np.ones(self.N)
            lin = np.zeros(self.N, dtype=np.int64)
            for a in range(self.ndim):
                w = w * self.wts[a][:, combo[a]]
                lin = lin * self.gshape[a] + self.taps[a][:, combo[a]]
            yield lin, w

    def interp(self, grid: np.ndarray) -> np.ndarray:
        """Sample value = sum over the W^ndim taps of phi-weight * grid value.
        ``grid`` has shape gshape + (C,); returns [N, C]."""
        C = grid.shape[-1]
        flat = grid.reshape(-1, C)
        out = np.zeros((self.N, C), dtype=np.complex128)
        for lin, w in self._tap_iter():
            out += w[:, None] * flat[lin]
        return out

    def spread(self, vals: np.ndarray) -> np.ndarray:
        """Adjoint of ``interp``: grid[g] = sum_i phi-weight(i, g) * vals[i]."""
        C = vals.shape[-1]
        M = int(np.prod(self.gshape))
        out = np.zeros((M, C), dtype=np.complex128)
        for lin, w in self._tap_iter():
            for c in range(C):
                out[:, c] += np.bincount(lin, weights=w * vals[:, c].real, minlength=M)
                out[:, c] += 1j * np.bincount(lin, weights=w * vals[:, c].imag, minlength=M)
        return out.reshape(self.gshape + (C,))

    # -- padding --------------------------------------------------------------
    def _pad(self, z: np.ndarray) -> np.ndarray:
        """Place image index i (centred r = i - n//2) at grid index r mod m."""
        C = z.shape[-1]
        g = np.zeros(self.gshape + (C,), dtype=np.complex128)
        idx = [np.mod(np.arange(n) - n // 2, m) for n, m in zip(self.shape, self.gshape)]
        g[np.ix_(*idx)] = z
        return g

    def _crop(self, g: np.ndarray) -> np.ndarray:
        idx = [np.mod(np.arange(n) - n // 2, m) for n, m in zip(self.shape, self.gshape)]
        return g[np.ix_(*idx)]

    # -- operators ----------------------------------------------------------
    def fft_grid(self, z: np.ndarray) -> np.ndarray:
        """Unnormalised oversampled DFT sum_r z[r] exp(-2 pi i g r / m)."""
        return np.fft.fftn(self._pad(z), axes=tuple(range(self.ndim)))

    def ifft_grid(self, g: np.ndarray) -> np.ndarray:
        """Adjoint of ``fft_grid``: sum_g G[g] exp(+2 pi i g r / m), cropped."""
        M = int(np.prod(self.gshape))
        return self._crop(np.fft.ifftn(g, axes=tuple(range(self.ndim))) * M)

    def forward(self, x: np.ndarray, maps: np.ndarray, weight: str = "sqrt") -> np.ndarray:
        """y_c = w^1/2 * NUFFT(c_c * x) (Eq. 5); returns [N, C]."""
        z = maps * (x / self.apod)[..., None]
        v = self.interp(self.fft_grid(z)) / math.sqrt(self.D)
        return v * self._w(weight)[:, None]

    def adjoint(self, y: np.ndarray, maps: np.ndarray, weight: str = "sqrt") -> np.ndarray:
        """x = sum_c conj(c_c) * NUFFT^H(w^1/2 * y_c)."""
        g = self.spread(y * self._w(weight)[:, None])
        z = self.ifft_grid(g) / math.sqrt(self.D)
        z = z / self.apod[..., None]
        return np.sum(np.conj(maps) * z, axis=-1)

    def normal(self, x: np.ndarray, maps: np.ndarray) -> np.ndarray:
        """A^H A x = sum_c conj(c_c) F^H W F (c_c x)."""
        z = maps * (x / self.apod)[..., None]
        v = self.interp(self.fft_grid(z)) / math.sqrt(self.D)
        v = v * self._w("full")[:, None]
        g = self.spread(v)
        out = self.ifft_grid(g) / math.sqrt(self.D) / self.apod[..., None]
        return np.sum(np.conj(maps) * out, axis=-1)

    def _w(self, kind: str) -> np.ndarray:
        if self.dcf is None:
            return np.ones(self.N)
        return np.sqrt(self.dcf) if kind == "sqrt" else self.dcf


def ndft_matrix(shape, coords) -> np.ndarray:
    """Brute-force NDFT matrix of Eq. 1 (rows = samples, columns = pixels in
    row-major order), including the 1/sqrt(D) factor."""
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    D = int(np.prod(shape))
    grids = np.meshgrid(*[np.arange(n) - n // 2 for n in shape], indexing="ij")
    phase = np.zeros((coords.shape[0], D))
    for a in range(ndim):
        r = grids[a].reshape(D)
        k = coords[:, ndim - 1 - a]
        phase += np.outer(k, r) / shape[a]
    return np.exp(-2j * np.pi * phase) / math.sqrt(D)


def ndft_forward(x, maps, coords, dcf=None):
    """Exact Eq. 1 (noise-free) with density compensation: [N, C]."""
    E = ndft_matrix(x.shape, coords)
    D = x.size
    z = (maps * x[..., None]).reshape(D, -1)
    y = E @ z
    if dcf is not None:
        y = y * np.sqrt(dcf)[:, None]
    return y
