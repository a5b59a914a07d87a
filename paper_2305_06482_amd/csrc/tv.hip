// l1 total variation (Sec. 2.1, regularizer 3): the periodic first-order
// difference operator T, (T x)_a[i] = x[i + e_a] - x[i] for every image axis
// a, and the two PDHG updates (Chambolle and Pock 2011) that touch it:
//   dual:   u_a <- clip(u_a + sigma (T xbar)_a, lambda)   (each complex
//           component projected onto the disc of radius lambda)
//   primal: v <- x - tau T^H u,  T^H u = sum_a (u_a[i - e_a] - u_a[i])
// Both are HBM-bound elementwise stencils: one thread per voxel, all axes.
#include <cmath>

#include "cs_internal.h"

namespace cs {

namespace {

struct Dims {
  int nz, ny, nx, ndim;  // nz = 1 in 2D
};

__device__ __forceinline__ void coords(long long i, const Dims& d, int& z, int& y, int& x) {
  x = (int)(i % d.nx);
  const long long r = i / d.nx;
  y = (int)(r % d.ny);
  z = (int)(r / d.ny);
}

__device__ __forceinline__ long long idx(int z, int y, int x, const Dims& d) {
  return ((long long)z * d.ny + y) * d.nx + x;
}

// component a of the axes in storage order: 3D (z, y, x), 2D (y, x)
__device__ __forceinline__ long long neighbour(int z, int y, int x, int a, int step,
                                               const Dims& d) {
  const int ax = d.ndim == 3 ? a : a + 1;  // 0 = z, 1 = y, 2 = x
  if (ax == 0) {
    int zz = z + step;
    zz = zz < 0 ? zz + d.nz : (zz >= d.nz ? zz - d.nz : zz);
    return idx(zz, y, x, d);
  }
  if (ax == 1) {
    int yy = y + step;
    yy = yy < 0 ? yy + d.ny : (yy >= d.ny ? yy - d.ny : yy);
    return idx(z, yy, x, d);
  }
  int xx = x + step;
  xx = xx < 0 ? xx + d.nx : (xx >= d.nx ? xx - d.nx : xx);
  return idx(z, y, xx, d);
}

__global__ void k_tv_dual(float2* __restrict__ u, const float2* __restrict__ xbar, float sigma,
                          float lam, Dims d, long long D) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  int z, y, x;
  coords(i, d, z, y, x);
  const float2 xi = xbar[i];
  for (int a = 0; a < d.ndim; ++a) {
    const float2 xn = xbar[neighbour(z, y, x, a, 1, d)];
    float2 w = u[(long long)a * D + i];
    w.x += sigma * (xn.x - xi.x);
    w.y += sigma * (xn.y - xi.y);
    const float m = sqrtf(w.x * w.x + w.y * w.y);
    const float s = m > lam ? lam / m : 1.f;
    u[(long long)a * D + i] = make_float2(w.x * s, w.y * s);
  }
}

__global__ void k_tv_primal(float2* __restrict__ v, const float2* __restrict__ xcur,
                            const float2* __restrict__ u, float tau, Dims d, long long D) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  int z, y, x;
  coords(i, d, z, y, x);
  float2 acc = make_float2(0.f, 0.f);
  for (int a = 0; a < d.ndim; ++a) {
    const float2 um = u[(long long)a * D + neighbour(z, y, x, a, -1, d)];
    const float2 ui = u[(long long)a * D + i];
    acc.x += um.x - ui.x;
    acc.y += um.y - ui.y;
  }
  const float2 xi = xcur[i];
  v[i] = make_float2(xi.x - tau * acc.x, xi.y - tau * acc.y);
}

Dims dims_of(const cs_ctx* c) {
  Dims d;
  d.ndim = c->ndim;
  d.nz = c->nz;
  d.ny = c->ny;
  d.nx = c->nx;
  return d;
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int tv_dual_step(cs_ctx* c, float2* u, const float2* xbar, float sigma, float lam) {
  CS_KLAUNCH(c, K_VEC, k_tv_dual, dim3(blocks_for(c->D)), dim3(256), 0, c->stream, u, xbar,
             sigma, lam, dims_of(c), c->D);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int tv_primal_step(cs_ctx* c, float2* v, const float2* x, const float2* u, float tau) {
  CS_KLAUNCH(c, K_VEC, k_tv_primal, dim3(blocks_for(c->D)), dim3(256), 0, c->stream, v, x, u,
             tau, dims_of(c), c->D);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

}  // namespace cs
