// Element-wise FISTA updates (FP32) and FP64 reductions in a fixed order.
//
// FISTA (Beck & Teboulle), the solver the paper uses for the l1-wavelet
// problem (Sec. 2.1.1) and for the sketched subproblems (Sec. 3.3.1):
//   v = z - alpha (g1 + s g2),  x+ = prox(v),  z = x+ + beta (x+ - x).
// Reductions accumulate in FP64: every block sums a fixed contiguous range in
// a fixed tree order, and a single block then sums the block partials in
// index order, so the result does not depend on scheduling.
#include <cmath>

#include "cs_internal.h"

namespace cs {

namespace {

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

__global__ void k_fill(float2* x, long long n, float re, float im) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) x[i] = make_float2(re, im);
}

__global__ void k_axpby(float2* out, float a, const float2* x, float b, const float2* y,
                        long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    const float2 u = x[i], v = y[i];
    out[i] = make_float2(a * u.x + b * v.x, a * u.y + b * v.y);
  }
}

__global__ void k_copy(float2* out, const float2* x, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) out[i] = x[i];
}

// v = z - alpha (g1 + s2 g2)
__global__ void k_fista_step(float2* v, const float2* z, float alpha, const float2* g1,
                             float s2, const float2* g2, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    const float2 a = g1[i], b = g2[i], zz = z[i];
    const float gx = a.x + s2 * b.x, gy = a.y + s2 * b.y;
    v[i] = make_float2(zz.x - alpha * gx, zz.y - alpha * gy);
  }
}

// z = xn + beta (xn - x); x = xn
__global__ void k_momentum(float2* z, float2* x, const float2* xn, float beta, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    const float2 a = xn[i], b = x[i];
    z[i] = make_float2(a.x + beta * (a.x - b.x), a.y + beta * (a.y - b.y));
    x[i] = a;
  }
}

// block partial sums of two FP64 quantities
// mode 0: conj(a) b (re, im);  mode 1: |a - b|^2, |b|^2;  mode 2: |a|, 0
__global__ __launch_bounds__(kRedThreads) void k_reduce_part(const float2* a,
                                                             const float2* b, long long n,
                                                             int mode, double* part) {
  __shared__ double s0[kRedThreads], s1[kRedThreads];
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = min(n, beg + per);
  double q0 = 0.0, q1 = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const float2 u = a[i], v = b[i];
    if (mode == 0) {
      q0 += (double)u.x * v.x + (double)u.y * v.y;
      q1 += (double)u.x * v.y - (double)u.y * v.x;
    } else if (mode == 2) {
      q0 += std::sqrt((double)u.x * u.x + (double)u.y * u.y);
    } else {
      const double dx = (double)u.x - v.x, dy = (double)u.y - v.y;
      q0 += dx * dx + dy * dy;
      q1 += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  s0[threadIdx.x] = q0;
  s1[threadIdx.x] = q1;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

// one block: thread t sums partials t, t + 256, ... in order, then a fixed
// tree over the threads
__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* part, int nparts,
                                                              double* out) {
  __shared__ double s0[kRedThreads], s1[kRedThreads];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kRedThreads) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

unsigned nblocks(long long n) {
  long long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

int reduce2(cs_ctx* c, const float2* a, const float2* b, long long n, int mode,
            double out[2]) {
  CS_KLAUNCH(c, K_REDUCE, k_reduce_part, dim3(kRedBlocks), dim3(kRedThreads), 0, c->stream, a, b,
                     n, mode, c->red);
  CS_KLAUNCH(c, K_REDUCE, k_reduce_final, dim3(1), dim3(kRedThreads), 0, c->stream, c->red,
             kRedBlocks, c->red_out);
  CS_HIP(c, hipGetLastError());
  CS_HIP(c, hipMemcpyAsync(c->host_red, c->red_out, 2 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  CS_HIP(c, hipStreamSynchronize(c->stream));
  out[0] = c->host_red[0];
  out[1] = c->host_red[1];
  return CS_OK;
}

}  // namespace

int vec_fill(cs_ctx* c, float2* x, long long n, float re, float im) {
  CS_KLAUNCH(c, K_VEC, k_fill, dim3(nblocks(n)), dim3(256), 0, c->stream, x, n, re, im);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int vec_axpby(cs_ctx* c, float2* out, float a, const float2* x, float b, const float2* y,
              long long n) {
  CS_KLAUNCH(c, K_VEC, k_axpby, dim3(nblocks(n)), dim3(256), 0, c->stream, out, a, x, b, y, n);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int vec_copy(cs_ctx* c, float2* out, const float2* x, long long n) {
  CS_KLAUNCH(c, K_VEC, k_copy, dim3(nblocks(n)), dim3(256), 0, c->stream, out, x, n);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int vec_fista_step(cs_ctx* c, float2* v, const float2* z, float alpha, const float2* g1,
                   float s2, const float2* g2, long long n) {
  CS_KLAUNCH(c, K_VEC, k_fista_step, dim3(nblocks(n)), dim3(256), 0, c->stream, v, z, alpha,
                     g1, s2, g2, n);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int vec_momentum(cs_ctx* c, float2* z, float2* x, const float2* xn, float beta,
                 long long n) {
  CS_KLAUNCH(c, K_VEC, k_momentum, dim3(nblocks(n)), dim3(256), 0, c->stream, z, x, xn, beta,
                     n);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int vec_dot(cs_ctx* c, const float2* a, const float2* b, long long n, double out[2]) {
  return reduce2(c, a, b, n, 0, out);
}

int vec_dist(cs_ctx* c, const float2* a, const float2* b, long long n, double* num,
             double* den) {
  double o[2];
  CS_TRY(reduce2(c, a, b, n, 1, o));
  *num = o[0];
  *den = o[1];
  return CS_OK;
}

int vec_abs_sum(cs_ctx* c, const float2* a, long long n, double* out) {
  double o[2];
  CS_TRY(reduce2(c, a, a, n, 2, o));
  *out = o[0];
  return CS_OK;
}

}  // namespace cs
