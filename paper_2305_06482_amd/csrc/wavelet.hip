// Unitary periodized Daubechies-4 wavelet transform and the l1-wavelet
// proximal step Psi^H soft(Psi v, tau) for g(x) = lambda ||Psi x||_1
// (Sec. 2.1, regularizer 2; "Daubechies 4" in Sec. 3.3.1).
//
// Filter: the 8-tap minimum-phase Daubechies scaling filter with four
// vanishing moments, obtained at start-up from the spectral factorisation
// |H(w)|^2 = 2 cos^8(w/2) P(sin^2(w/2)), P(y) = 1 + 4y + 10y^2 + 20y^3: the
// roots of P are found by Durand-Kerner iteration, each gives the root of
// zeta^2 - (2 - 4y) zeta + 1 = 0 outside the unit circle, and
// H(zeta) = (1 + zeta)^4 prod (zeta - zeta_r) is normalised to sum h = sqrt 2.
//
// One level along an axis of (even) length L:
//   a[k] = sum_n h[n] x[(2k + n) mod L],  d[k] = sum_n g[n] x[(2k + n) mod L],
//   g[n] = (-1)^n h[7 - n], output [a, d];
// levels recurse on the approximation block (Mallat layout), and the inverse
// is the transpose.  Soft threshold: w max(0, 1 - tau / |w|).
#include <cmath>
#include <complex>

#include "cs_internal.h"

namespace cs {

namespace {

__constant__ float c_h[8];
__constant__ float c_g[8];

using cd = std::complex<double>;

// roots of the monic-normalised polynomial with ascending coefficients a[0..n]
std::vector<cd> poly_roots(const std::vector<double>& a) {
  const int n = (int)a.size() - 1;
  std::vector<cd> z(n);
  const cd seed(0.4, 0.9);
  for (int i = 0; i < n; ++i) z[i] = std::pow(seed, i);
  auto eval = [&](cd x) {
    cd v = a[n];
    for (int k = n - 1; k >= 0; --k) v = v * x + a[k];
    return v / a[n];
  };
  for (int it = 0; it < 500; ++it) {
    double delta = 0.0;
    for (int i = 0; i < n; ++i) {
      cd den = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != i) den *= (z[i] - z[j]);
      const cd step = eval(z[i]) / den;
      z[i] -= step;
      delta = std::max(delta, std::abs(step));
    }
    if (delta < 1e-15) break;
  }
  return z;
}

void daubechies4(double h[8]) {
  const int p = 4;
  std::vector<double> P(p);
  // binomial(p - 1 + k, k)
  for (int k = 0; k < p; ++k) {
    double b = 1.0;
    for (int i = 1; i <= k; ++i) b = b * (double)(p - 1 + i) / (double)i;
    P[k] = b;
  }
  std::vector<cd> yr = poly_roots(P);
  std::vector<cd> poly = {cd(1.0)};  // ascending powers of zeta
  auto mul = [&](cd r0, cd r1) {      // poly *= (r0 + r1 zeta)
    std::vector<cd> out(poly.size() + 1, cd(0.0));
    for (size_t i = 0; i < poly.size(); ++i) {
      out[i] += poly[i] * r0;
      out[i + 1] += poly[i] * r1;
    }
    poly = out;
  };
  for (int i = 0; i < p; ++i) mul(1.0, 1.0);
  for (const cd& y : yr) {
    const cd b = 2.0 - 4.0 * y;
    const cd disc = std::sqrt(b * b - 4.0);
    const cd z1 = (b + disc) / 2.0, z2 = (b - disc) / 2.0;
    const cd zr = std::abs(z1) > 1.0 ? z1 : z2;
    mul(-zr, 1.0);
  }
  double s = 0.0;
  for (int i = 0; i < 2 * p; ++i) s += poly[i].real();
  for (int i = 0; i < 2 * p; ++i) h[i] = poly[i].real() * std::sqrt(2.0) / s;
}

// one analysis level along `axis` of the region [rz][ry][rx] of an array with
// row-major extents (nz, ny, nx): src -> dst
__global__ void k_dwt_axis(const float2* __restrict__ src, float2* __restrict__ dst, int ny,
                           int nx, int rz, int ry, int rx, int axis) {
  const long long total = (long long)rz * ry * rx;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int x = (int)(i % rx);
  const int y = (int)((i / rx) % ry);
  const int z = (int)(i / ((long long)rx * ry));
  const int L = axis == 2 ? rx : (axis == 1 ? ry : rz);
  const int pos = axis == 2 ? x : (axis == 1 ? y : z);
  const long long stride = axis == 2 ? 1 : (axis == 1 ? nx : (long long)ny * nx);
  const long long base = ((long long)z * ny + y) * nx + x - (long long)pos * stride;
  const int half = L / 2;
  const bool det = pos >= half;
  const int k = det ? pos - half : pos;
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    int q = (2 * k + n) % L;
    const float2 v = src[base + (long long)q * stride];
    const float f = det ? c_g[n] : c_h[n];
    acc.x += f * v.x;
    acc.y += f * v.y;
  }
  dst[base + (long long)pos * stride] = acc;
}

// transpose of k_dwt_axis: x[m] = sum_{n = m mod 2 + 2i} h[n] a[(m-n)/2] + g[n] d[(m-n)/2]
__global__ void k_idwt_axis(const float2* __restrict__ src, float2* __restrict__ dst, int ny,
                            int nx, int rz, int ry, int rx, int axis) {
  const long long total = (long long)rz * ry * rx;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int x = (int)(i % rx);
  const int y = (int)((i / rx) % ry);
  const int z = (int)(i / ((long long)rx * ry));
  const int L = axis == 2 ? rx : (axis == 1 ? ry : rz);
  const int m = axis == 2 ? x : (axis == 1 ? y : z);
  const long long stride = axis == 2 ? 1 : (axis == 1 ? nx : (long long)ny * nx);
  const long long base = ((long long)z * ny + y) * nx + x - (long long)m * stride;
  const int half = L / 2;
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = (m & 1) + 2 * q;
    int k = ((m - n) / 2) % half;
    if (k < 0) k += half;
    const float2 a = src[base + (long long)k * stride];
    const float2 d = src[base + (long long)(k + half) * stride];
    acc.x += c_h[n] * a.x + c_g[n] * d.x;
    acc.y += c_h[n] * a.y + c_g[n] * d.y;
  }
  dst[base + (long long)m * stride] = acc;
}

__global__ void k_copy_region(const float2* __restrict__ src, float2* __restrict__ dst,
                              int ny, int nx, int rz, int ry, int rx) {
  const long long total = (long long)rz * ry * rx;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int x = (int)(i % rx);
  const int y = (int)((i / rx) % ry);
  const int z = (int)(i / ((long long)rx * ry));
  const long long o = ((long long)z * ny + y) * nx + x;
  dst[o] = src[o];
}

__global__ void k_soft(float2* __restrict__ w, long long n, float tau) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    const float2 v = w[i];
    const float mag = sqrtf(v.x * v.x + v.y * v.y);
    const float s = mag > tau ? 1.f - tau / mag : 0.f;
    w[i] = make_float2(v.x * s, v.y * s);
  }
}

unsigned nb(long long n) { return (unsigned)((n + 255) / 256); }

int axis_pass(cs_ctx* c, bool inv, const float2* src, float2* dst, int rz, int ry, int rx,
              int axis) {
  const long long total = (long long)rz * ry * rx;
  if (inv)
    CS_KLAUNCH(c, K_WAVELET, k_idwt_axis, dim3(nb(total)), dim3(256), 0, c->stream, src, dst, c->ny,
                       c->nx, rz, ry, rx, axis);
  else
    CS_KLAUNCH(c, K_WAVELET, k_dwt_axis, dim3(nb(total)), dim3(256), 0, c->stream, src, dst, c->ny,
                       c->nx, rz, ry, rx, axis);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int copy_region(cs_ctx* c, const float2* src, float2* dst, int rz, int ry, int rx) {
  const long long total = (long long)rz * ry * rx;
  CS_KLAUNCH(c, K_WAVELET, k_copy_region, dim3(nb(total)), dim3(256), 0, c->stream, src, dst, c->ny,
                     c->nx, rz, ry, rx);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

// levels of the transform over buffer `w` (in place), using `t` as scratch
int dwt_levels(cs_ctx* c, float2* w, float2* t, bool inv) {
  const int Lv = c->g.wav_levels;
  int sz[16][3];
  int rz = c->nz, ry = c->ny, rx = c->nx;
  for (int l = 0; l < Lv; ++l) {
    sz[l][0] = rz; sz[l][1] = ry; sz[l][2] = rx;
    if (c->ndim == 3) rz /= 2;
    ry /= 2;
    rx /= 2;
  }
  for (int s = 0; s < Lv; ++s) {
    const int l = inv ? Lv - 1 - s : s;
    const int z = sz[l][0], y = sz[l][1], x = sz[l][2];
    if (!inv) {
      // x, then y, then z (3D)
      CS_TRY(axis_pass(c, false, w, t, z, y, x, 2));
      CS_TRY(axis_pass(c, false, t, w, z, y, x, 1));
      if (c->ndim == 3) {
        CS_TRY(axis_pass(c, false, w, t, z, y, x, 0));
        CS_TRY(copy_region(c, t, w, z, y, x));
      }
    } else {
      // reverse order: z, y, x
      if (c->ndim == 3) {
        CS_TRY(axis_pass(c, true, w, t, z, y, x, 0));
        CS_TRY(axis_pass(c, true, t, w, z, y, x, 1));
        CS_TRY(axis_pass(c, true, w, t, z, y, x, 2));
        CS_TRY(copy_region(c, t, w, z, y, x));
      } else {
        CS_TRY(axis_pass(c, true, w, t, z, y, x, 1));
        CS_TRY(axis_pass(c, true, t, w, z, y, x, 2));
      }
    }
  }
  return CS_OK;
}

}  // namespace

int wavelet_init(cs_ctx* c) {
  double h[8];
  daubechies4(h);
  float hf[8], gf[8];
  for (int n = 0; n < 8; ++n) {
    hf[n] = (float)h[n];
    gf[n] = (float)(((n & 1) ? -1.0 : 1.0) * h[7 - n]);
  }
  CS_HIP(c, hipMemcpyToSymbol(HIP_SYMBOL(c_h), hf, sizeof(hf)));
  CS_HIP(c, hipMemcpyToSymbol(HIP_SYMBOL(c_g), gf, sizeof(gf)));
  return CS_OK;
}

int dwt_fwd(cs_ctx* c, const float2* x, float2* coef) {
  CS_TRY(vec_copy(c, coef, x, c->D));
  return dwt_levels(c, coef, c->wav2, false);
}

int dwt_inv(cs_ctx* c, const float2* coef, float2* x) {
  CS_TRY(vec_copy(c, x, coef, c->D));
  return dwt_levels(c, x, c->wav2, true);
}

int prox_l1(cs_ctx* c, const float2* v, float tau, float2* out) {
  CS_TRY(vec_copy(c, c->wav1, v, c->D));
  CS_TRY(dwt_levels(c, c->wav1, c->wav2, false));
  CS_KLAUNCH(c, K_SOFT, k_soft, dim3(std::min<long long>(8192, nb(c->D))), dim3(256), 0,
                     c->stream, c->wav1, c->D, tau);
  CS_HIP(c, hipGetLastError());
  CS_TRY(dwt_levels(c, c->wav1, c->wav2, true));
  return vec_copy(c, out, c->wav1, c->D);
}

}  // namespace cs
