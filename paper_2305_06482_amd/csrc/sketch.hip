// Structured coil sketch (Sec. 2.3.2-2.3.3, Eqs. 11-13).
//
//  1. Coil covariance R = sum_i k_i k_i^H of the raw samples k_i = y_i / sqrt(w_i)
//     (PCA coil compression, Alg. 1 and Sec. 3.1), accumulated in FP64:
//     each block sums a fixed range of samples, then the block partials are
//     summed in index order.
//  2. R = U diag(lambda) U^H by cyclic complex Jacobi rotations in FP64 in one
//     work-group; eigenvalues sorted descending (index order on ties) and the
//     largest-magnitude entry of each eigenvector made real positive.
//  3. Coil mixing out[d][j] = sum_c in[d][c] M[j][c] at every pixel d (Eq. 13),
//     as a real GEMM over interleaved (re, im) columns on MFMA
//     (v_mfma_f32_16x16x16_bf16, FP32 accumulate).  FP32 operands are split
//     into bf16 terms hi + mid + lo (round-to-nearest-even each), and the
//     products with combined order below three are summed, which keeps the
//     result at FP32 accuracy.  The +-1 Rademacher entries are exact in bf16,
//     so the per-iteration sketch needs only the three products of the split
//     maps with them; the 1/sqrt(S) scale is applied in FP32 in the epilogue.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "cs_internal.h"

namespace cs {

namespace {

constexpr int kCovBlocks = 512;
constexpr int kCovChunk = 32;     // samples staged in LDS per step
constexpr int kMaxC = 64;

// ---- 1. covariance ---------------------------------------------------------
__global__ __launch_bounds__(256) void k_cov_part(const float2* __restrict__ y, int C,
                                                  const float* __restrict__ dcf,
                                                  long long N, double* __restrict__ part) {
  __shared__ double2 ks[kCovChunk * kMaxC];
  const long long per = (N + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * per;
  const long long end = min(N, beg + per);
  const int CC = C * C;
  constexpr int kAcc = kMaxC * kMaxC / 256;
  double2 acc[kAcc];
  int ea[kAcc], eb[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) {
    acc[q] = make_double2(0.0, 0.0);
    const int e = threadIdx.x + q * 256;
    ea[q] = e < CC ? e / C : 0;
    eb[q] = e < CC ? e % C : 0;
  }
  for (long long s0 = beg; s0 < end; s0 += kCovChunk) {
    const int ns = (int)min((long long)kCovChunk, end - s0);
    __syncthreads();
    for (int i = threadIdx.x; i < ns * C; i += blockDim.x) {
      const int s = i / C, c = i % C;
      const long long smp = s0 + s;
      const float2 v = y[smp * C + c];
      double sc = 1.0;
      if (dcf) {
        const float w = dcf[smp];
        sc = w > 0.f ? 1.0 / sqrt((double)w) : 0.0;
      }
      ks[s * C + c] = make_double2(v.x * sc, v.y * sc);
    }
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
#pragma unroll
      for (int q = 0; q < kAcc; ++q) {
        if (threadIdx.x + q * 256 < CC) {
          const double2 ka = ks[s * C + ea[q]], kb = ks[s * C + eb[q]];
          // k_a conj(k_b)
          acc[q].x += ka.x * kb.x + ka.y * kb.y;
          acc[q].y += ka.y * kb.x - ka.x * kb.y;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kAcc; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < CC) {
      part[((long long)blockIdx.x * CC + e) * 2] = acc[q].x;
      part[((long long)blockIdx.x * CC + e) * 2 + 1] = acc[q].y;
    }
  }
}

__global__ void k_cov_final(const double* __restrict__ part, int nparts, int CC,
                            double* __restrict__ R) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= CC) return;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < nparts; ++p) {
    re += part[((long long)p * CC + e) * 2];
    im += part[((long long)p * CC + e) * 2 + 1];
  }
  R[2 * e] = re;
  R[2 * e + 1] = im;
}

// ---- 2. Jacobi eigensolver ------------------------------------------------
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}

// out: U [C][C] complex (re, im) row-major, then lambda [C]
__global__ __launch_bounds__(64) void k_jacobi(const double* __restrict__ Rin, int C,
                                               double* __restrict__ out) {
  extern __shared__ double2 sh[];
  double2* A = sh;            // [C][C]
  double2* V = sh + C * C;    // [C][C]
  __shared__ double2 G[4];    // Gpp, Gpq, Gqp, Gqq
  __shared__ int go;
  __shared__ double offn, diagn;
  __shared__ int order[kMaxC];
  const int tid = threadIdx.x;
  for (int i = tid; i < C * C; i += blockDim.x) {
    A[i] = make_double2(Rin[2 * i], Rin[2 * i + 1]);
    V[i] = make_double2((i / C) == (i % C) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) {
      double o = 0.0, d = 0.0;
      for (int p = 0; p < C; ++p) {
        d += A[p * C + p].x * A[p * C + p].x;
        for (int q = p + 1; q < C; ++q)
          o += A[p * C + q].x * A[p * C + q].x + A[p * C + q].y * A[p * C + q].y;
      }
      offn = o;
      diagn = d;
    }
    __syncthreads();
    if (offn <= 1e-32 * diagn || offn == 0.0) break;
    for (int p = 0; p < C - 1; ++p) {
      for (int q = p + 1; q < C; ++q) {
        if (tid == 0) {
          const double2 apq = A[p * C + q];
          const double r = sqrt(apq.x * apq.x + apq.y * apq.y);
          const double a = A[p * C + p].x, b = A[q * C + q].x;
          go = r > 1e-300 && r > 1e-18 * sqrt(fabs(a * b));
          if (go) {
            // unit phase e^{i phi} = apq / r; rotation zeroing the real pair
            const double2 ph = make_double2(apq.x / r, apq.y / r);
            const double theta = (b - a) / (2.0 * r);
            const double t = (theta >= 0 ? 1.0 : -1.0) /
                             (fabs(theta) + sqrt(theta * theta + 1.0));
            const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
            const double2 em = zconj(ph);  // e^{-i phi}
            G[0] = make_double2(cs, 0.0);
            G[1] = make_double2(sn, 0.0);
            G[2] = make_double2(-sn * em.x, -sn * em.y);
            G[3] = make_double2(cs * em.x, cs * em.y);
          }
        }
        __syncthreads();
        if (go) {
          const double2 g0 = G[0], g1 = G[1], g2 = G[2], g3 = G[3];
          // A <- A G and V <- V G (columns p, q)
          for (int k = tid; k < C; k += blockDim.x) {
            const double2 akp = A[k * C + p], akq = A[k * C + q];
            A[k * C + p] = zadd(zmul(akp, g0), zmul(akq, g2));
            A[k * C + q] = zadd(zmul(akp, g1), zmul(akq, g3));
            const double2 vkp = V[k * C + p], vkq = V[k * C + q];
            V[k * C + p] = zadd(zmul(vkp, g0), zmul(vkq, g2));
            V[k * C + q] = zadd(zmul(vkp, g1), zmul(vkq, g3));
          }
          __syncthreads();
          // A <- G^H A (rows p, q)
          for (int k = tid; k < C; k += blockDim.x) {
            const double2 apk = A[p * C + k], aqk = A[q * C + k];
            A[p * C + k] = zadd(zmul(zconj(g0), apk), zmul(zconj(g2), aqk));
            A[q * C + k] = zadd(zmul(zconj(g1), apk), zmul(zconj(g3), aqk));
          }
          __syncthreads();
          if (tid == 0) {
            A[p * C + q] = make_double2(0.0, 0.0);
            A[q * C + p] = make_double2(0.0, 0.0);
            A[p * C + p].y = 0.0;
            A[q * C + q].y = 0.0;
          }
          __syncthreads();
        }
      }
    }
  }
  // sort descending by eigenvalue (stable in index), fix phases
  if (tid == 0) {
    for (int i = 0; i < C; ++i) order[i] = i;
    for (int i = 1; i < C; ++i) {
      const int v = order[i];
      int j = i - 1;
      while (j >= 0 && A[order[j] * C + order[j]].x < A[v * C + v].x) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = v;
    }
  }
  __syncthreads();
  for (int jj = tid; jj < C; jj += blockDim.x) {
    const int j = order[jj];
    int imax = 0;
    double best = -1.0;
    for (int i = 0; i < C; ++i) {
      const double2 v = V[i * C + j];
      const double m = v.x * v.x + v.y * v.y;
      if (m > best) {
        best = m;
        imax = i;
      }
    }
    const double2 u = V[imax * C + j];
    const double mu = sqrt(u.x * u.x + u.y * u.y);
    const double2 ph = make_double2(u.x / mu, -u.y / mu);  // conj(u) / |u|
    for (int i = 0; i < C; ++i) {
      double2 v = zmul(V[i * C + j], ph);
      if (i == imax) v.y = 0.0;
      out[2 * (i * C + jj)] = v.x;
      out[2 * (i * C + jj) + 1] = v.y;
    }
    out[2 * C * C + jj] = A[j * C + j].x;
  }
}

// ---- 3. coil mixing on MFMA -------------------------------------------------
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

// A: [D] rows of cin complex (row d at in + d*in_ldc + in_c0), K = 2 cin
// B fragments: [nB terms][nK][nN][64 lanes][4] bf16, prepared on the host
// out: row d at out + d*out_ldc + out_c0, N = 2 cout columns
__global__ __launch_bounds__(256) void k_coil_mix(const float2* __restrict__ in, int in_ldc,
                                                  int in_c0, int cin, long long D,
                                                  const v4s* __restrict__ Bf, int nB, int nK,
                                                  int nN, float2* __restrict__ out,
                                                  int out_ldc, int out_c0, int cout,
                                                  float scale) {
  const int lane = threadIdx.x & 63;
  const long long tile = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const long long d0 = tile * 16;
  if (d0 >= D) return;
  const int row = lane & 15;      // A row within the tile
  const int kq = lane >> 4;       // which 4-group of K
  const long long d = d0 + row;
  const bool rowok = d < D;
  const int K = 2 * cin;
  v4f acc[8];
  for (int n = 0; n < nN; ++n) acc[n] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < nK; ++kb) {
    float a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = kb * 16 + kq * 4 + e;
      float v = 0.f;
      if (rowok && k < K) {
        const float2 z = in[d * in_ldc + in_c0 + (k >> 1)];
        v = (k & 1) ? z.y : z.x;
      }
      a[e] = v;
    }
    v4s ah, am, al;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned short h = bf16_rne(a[e]);
      const float r1 = a[e] - bf16_to_f(h);
      const unsigned short m = bf16_rne(r1);
      const float r2 = r1 - bf16_to_f(m);
      const unsigned short l = bf16_rne(r2);
      ah[e] = (short)h;
      am[e] = (short)m;
      al[e] = (short)l;
    }
    for (int n = 0; n < nN; ++n) {
      const v4s bh = Bf[((0 * nK + kb) * nN + n) * 64 + lane];
      v4f c = acc[n];
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, c, 0, 0, 0);
      if (nB > 1) {
        const v4s bm = Bf[((1 * nK + kb) * nN + n) * 64 + lane];
        const v4s bl = Bf[((2 * nK + kb) * nN + n) * 64 + lane];
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, c, 0, 0, 0);
      }
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
      acc[n] = c;
    }
  }
  // D[i][j]: lane holds column j = lane % 16 of rows i = 4 (lane / 16) + v
  const int N2 = 2 * cout;
  for (int n = 0; n < nN; ++n) {
    const int col = n * 16 + (lane & 15);
    if (col >= N2) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long dd = d0 + 4 * (lane >> 4) + v;
      if (dd < D) {
        float* o = reinterpret_cast<float*>(out + dd * out_ldc + out_c0);
        o[col] = acc[n][v] * scale;
      }
    }
  }
}

// Packs the B fragments of k_coil_mix from a mixing matrix in device memory
// (complex128 [cout][cin], row-major) exactly as coil_mix_rows packs them on
// the host: real B[k][n] with k = 2 cc + (0: re, 1: im of input coil cc) and
// n = 2 j + (0: re, 1: im of output coil j), i.e. B(2cc, 2j) = re M[j][cc],
// B(2cc+1, 2j) = -im, B(2cc, 2j+1) = im, B(2cc+1, 2j+1) = re, split into the
// three bf16 terms hi, mid, lo.  One thread per fragment element; every
// element of the nK x nN blocks of all three terms is written.
__global__ __launch_bounds__(256) void k_pack_mix(const double2* __restrict__ M, int cin,
                                                  int cout, int nK, int nN,
                                                  unsigned short* __restrict__ frag) {
  const int total = nK * nN * 64 * 4;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int e = i & 3, l = (i >> 2) & 63, blk = i >> 8;
  const int n = blk % nN, kb = blk / nN;
  const int k = kb * 16 + 4 * (l >> 4) + e, col = n * 16 + (l & 15);
  float v = 0.f;
  if (k < 2 * cin && col < 2 * cout) {
    const double2 m = M[(size_t)(col >> 1) * cin + (k >> 1)];
    const float re = (float)m.x, im = (float)m.y;
    v = (k & 1) == 0 ? ((col & 1) == 0 ? re : im) : ((col & 1) == 0 ? -im : re);
  }
  const unsigned short h = bf16_rne(v);
  const float r1 = v - bf16_to_f(h);
  const unsigned short mid = bf16_rne(r1);
  const float r2 = r1 - bf16_to_f(mid);
  const unsigned short lo = bf16_rne(r2);
  frag[i] = h;
  frag[total + i] = mid;
  frag[2 * total + i] = lo;
}

// Fragment scratch of the allocation-free coil mixing: the three split terms
// of the largest mixing matrix (64 x 64 complex: K = N = 128 real columns,
// 8 x 8 fragment blocks of 64 lanes x 4 bf16), 96 KiB.  Each GPU that loads
// the library holds one copy until the process ends; in host code the name
// stands for no device address, so host code uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr int kMixBlocksMax = 8;
constexpr size_t kMixFragElems = (size_t)3 * kMixBlocksMax * kMixBlocksMax * 64 * 4;
static __device__ __align__(256) unsigned short scratch[kMixFragElems];

unsigned short host_bf16(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
float host_bf16_f(unsigned short h) {
  unsigned u = (unsigned)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace

int covariance_eig(cs_ctx* c, const float2* y) {
  const int C = c->C;
  if (C > kMaxC) return fail(c, CS_EUNSUPPORTED, "more than 64 coils");
  const long long N = c->N;
  const float* dcf = c->g.kind == CS_NONCART ? c->dcf_orig : nullptr;
  CS_KLAUNCH(c, K_COV, k_cov_part, dim3(kCovBlocks), dim3(256), 0, c->stream, y, C, dcf, N,
                     c->cov_part);
  const int CC = C * C;
  CS_KLAUNCH(c, K_COV, k_cov_final, dim3((CC + 255) / 256), dim3(256), 0, c->stream,
                     c->cov_part, kCovBlocks, CC, c->cov);
  const size_t lds = sizeof(double2) * 2 * CC;
  CS_KLAUNCH(c, K_EIG, k_jacobi, dim3(1), dim3(64), lds, c->stream, c->cov, C, c->eig_dev);
  CS_HIP(c, hipGetLastError());
  std::vector<double> h((size_t)2 * CC + C);
  CS_HIP(c, hipMemcpyAsync(h.data(), c->eig_dev, sizeof(double) * h.size(),
                           hipMemcpyDeviceToHost, c->stream));
  CS_HIP(c, hipStreamSynchronize(c->stream));
  c->U.assign(h.begin(), h.begin() + 2 * CC);
  c->lam.assign(h.begin() + 2 * CC, h.end());
  for (double v : c->lam)
    if (!std::isfinite(v)) return fail(c, CS_ENUMERIC, "non-finite eigenvalue");
  return CS_OK;
}

int coil_mix(cs_ctx* c, const float2* in, int in_ldc, int in_c0, int cin, const double* M,
             int cout, float2* out, int out_ldc, int out_c0, float out_scale) {
  return coil_mix_rows(c, c->D, in, in_ldc, in_c0, cin, M, cout, out, out_ldc, out_c0,
                       out_scale);
}

// fragment buffer and pinned staging ring sized for the largest mixing
// matrix (64 x 64), so that coil mixing never allocates
int coil_mix_reserve(cs_ctx* c) {
  const size_t bytes = (size_t)3 * 8 * 8 * 64 * 4 * sizeof(unsigned short);
  CS_HIP(c, hipMalloc(&c->mixB, bytes));
  c->mixB_bytes = bytes;
  for (int k = 0; k < cs_ctx::kStage; ++k) {
    CS_HIP(c, hipHostMalloc(&c->stage[k], bytes, 0));
    c->stage_bytes[k] = bytes;
    CS_HIP(c, hipEventCreateWithFlags(&c->stage_ev[k], hipEventDisableTiming));
  }
  return CS_OK;
}

int coil_mix_rows(cs_ctx* c, long long rows, const float2* in, int in_ldc, int in_c0, int cin,
                  const double* M, int cout, float2* out, int out_ldc, int out_c0,
                  float out_scale) {
  if (cin < 1 || cout < 1 || cin > kMaxC || cout > 64)
    return fail(c, CS_EINVAL, "coil_mix sizes");
  const int K = 2 * cin, N2 = 2 * cout;
  const int nK = (K + 15) / 16, nN = (N2 + 15) / 16;
  if (nN > 8) return fail(c, CS_EINVAL, "coil_mix: too many output coils");
  // real B [K][N2] from complex M[j][c]
  std::vector<float> B((size_t)nK * 16 * nN * 16, 0.f);
  auto Bat = [&](int k, int n) -> float& { return B[(size_t)k * nN * 16 + n]; };
  bool exact = true;
  for (int j = 0; j < cout; ++j)
    for (int cc = 0; cc < cin; ++cc) {
      const float re = (float)M[2 * (j * cin + cc)], im = (float)M[2 * (j * cin + cc) + 1];
      Bat(2 * cc, 2 * j) = re;
      Bat(2 * cc + 1, 2 * j) = -im;
      Bat(2 * cc, 2 * j + 1) = im;
      Bat(2 * cc + 1, 2 * j + 1) = re;
    }
  for (float v : B)
    if (host_bf16_f(host_bf16(v)) != v) exact = false;
  const int nB = exact ? 1 : 3;
  // fragments: lane l holds B[kb*16 + 4 (l/16) + e][n*16 + l%16], e = 0..3
  std::vector<unsigned short> frag((size_t)3 * nK * nN * 64 * 4, 0);
  for (int kb = 0; kb < nK; ++kb)
    for (int n = 0; n < nN; ++n)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 4; ++e) {
          const float v = Bat(kb * 16 + 4 * (l / 16) + e, n * 16 + l % 16);
          const unsigned short h = host_bf16(v);
          const float r1 = v - host_bf16_f(h);
          const unsigned short m = host_bf16(r1);
          const float r2 = r1 - host_bf16_f(m);
          const unsigned short lo = host_bf16(r2);
          const size_t base = (((size_t)kb * nN + n) * 64 + l) * 4 + e;
          const size_t term = (size_t)nK * nN * 64 * 4;
          frag[base] = h;
          frag[term + base] = m;
          frag[2 * term + base] = lo;
        }
  const size_t bytes = frag.size() * sizeof(unsigned short);
  if (bytes > c->mixB_bytes || bytes > c->stage_bytes[c->stage_next])
    return fail(c, CS_EINVAL, "coil_mix: fragments exceed the reserved buffers");
  // stage through a pinned ring slot whose previous copy has completed (no
  // stream-wide synchronisation)
  const int k = c->stage_next;
  c->stage_next = (k + 1) % cs_ctx::kStage;
  CS_HIP(c, hipEventSynchronize(c->stage_ev[k]));
  std::memcpy(c->stage[k], frag.data(), bytes);
  CS_HIP(c, hipMemcpyAsync(c->mixB, c->stage[k], bytes, hipMemcpyHostToDevice, c->stream));
  CS_HIP(c, hipEventRecord(c->stage_ev[k], c->stream));
  if (rows <= 0) return CS_OK;
  const long long tiles = (rows + 15) / 16;
  const unsigned nb = (unsigned)((tiles + 3) / 4);
  CS_KLAUNCH(c, K_MIX, k_coil_mix, dim3(nb), dim3(256), 0, c->stream, in, in_ldc, in_c0, cin,
                     rows, (const v4s*)c->mixB, nB, nK, nN, out, out_ldc, out_c0, cout,
                     out_scale);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int mix_scratch_init(cs_ctx* c) {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device ordinal -> address of `scratch`
  int dev = -1;
  CS_HIP(c, hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    CS_HIP(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(c, CS_EHIP, "no device address for the coil-mixing scratch");
    it = addr.emplace(dev, p).first;
  }
  c->mix_scratch = it->second;
  return CS_OK;
}

int coil_mix_noalloc(cs_ctx* c, const float2* in, int cin, const void* M, int cout,
                     float2* out) {
  if (cin < 1 || cout < 1 || cin > kMixBlocksMax * 8 || cout > kMixBlocksMax * 8)
    return fail(c, CS_EINVAL,
                "cs_coil_mix_noalloc: cin and cout must be in [1, 64] (the scratch holds the "
                "fragments of a 64 x 64 mixing matrix at most)");
  if (!c->mix_scratch) return fail(c, CS_EHIP, "coil-mixing scratch address not set up");
  const int nK = (2 * cin + 15) / 16, nN = (2 * cout + 15) / 16;
  const int total = nK * nN * 64 * 4;
  auto* frag = (unsigned short*)c->mix_scratch;
  CS_KLAUNCH(c, K_MIX, k_pack_mix, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
             c->stream, (const double2*)M, cin, cout, nK, nN, frag);
  CS_HIP(c, hipGetLastError());
  const long long rows = c->D;
  if (rows <= 0) return CS_OK;
  const long long tiles = (rows + 15) / 16;
  const unsigned nb = (unsigned)((tiles + 3) / 4);
  CS_KLAUNCH(c, K_MIX, k_coil_mix, dim3(nb), dim3(256), 0, c->stream, in, cin, 0, cin, rows,
             (const v4s*)frag, 3, nK, nN, out, cout, 0, cout, 1.0f);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

}  // namespace cs
