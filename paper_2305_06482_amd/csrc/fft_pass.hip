// Batched mixed-radix FFT passes over LDS panels, with the sensitivity
// multiply / deapodisation / zero-padding fused into the first pass and the
// conjugate-map coil reduction fused into the last one (Sec. 2.1, Eqs. 2 and
// 5; Eq. 12 for the sketched maps).
//
// The FFT is a Stockham autosort transform: for radix R and current span Ns,
// butterfly j reads rows j + r L/R, multiplies element r by the twiddle
// e^{-2 pi i (j mod Ns) r / (Ns R)}, takes the R-point DFT and writes rows
// (j / Ns) Ns R + (j mod Ns) + r Ns.  Radices 2, 3, 4 and 5 cover every
// length of the form 2^a 3^b 5^c.
#include <cmath>

#include "cs_internal.h"

namespace cs {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) {
  return make_float2(a.x * s, a.y * s);
}
// a s, then + b when add: each product and sum rounded on its own (no fused
// multiply-add), so that every thread mapping of a pass gives the same bits
__device__ __forceinline__ float2 cscale_add(float2 a, float s, bool add, float2 b) {
  float2 r = make_float2(__fmul_rn(a.x, s), __fmul_rn(a.y, s));
  if (add) r = make_float2(__fadd_rn(r.x, b.x), __fadd_rn(r.y, b.y));
  return r;
}
// multiply by -i (dir < 0) or +i (dir > 0)
__device__ __forceinline__ float2 mul_i(float2 a, int dir) {
  return dir < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// cos / sin of 2 pi / 3 and 2 pi / 5, 4 pi / 5
constexpr float kS3 = 0.86602540378443864676f;
constexpr float kC51 = 0.30901699437494742410f;
constexpr float kC52 = -0.80901699437494742410f;
constexpr float kS51 = 0.95105651629515357212f;
constexpr float kS52 = 0.58778525229247312917f;

__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void dft3(float2* v, int dir) {
  float2 t1 = cadd(v[1], v[2]);
  float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  float2 t3 = mul_i(cscale(csub(v[1], v[2]), kS3), dir);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}

__device__ __forceinline__ void dft4(float2* v, int dir) {
  float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  float2 c = cadd(v[1], v[3]), d = mul_i(csub(v[1], v[3]), dir);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}

__device__ __forceinline__ void dft5(float2* v, int dir) {
  float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  float2 x0 = v[0];
  float2 r1 = make_float2(x0.x + kC51 * a1.x + kC52 * a2.x, x0.y + kC51 * a1.y + kC52 * a2.y);
  float2 r2 = make_float2(x0.x + kC52 * a1.x + kC51 * a2.x, x0.y + kC52 * a1.y + kC51 * a2.y);
  float2 i1 = mul_i(make_float2(kS51 * b1.x + kS52 * b2.x, kS51 * b1.y + kS52 * b2.y), dir);
  float2 i2 = mul_i(make_float2(kS52 * b1.x - kS51 * b2.x, kS52 * b1.y - kS51 * b2.y), dir);
  v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  v[1] = cadd(r1, i1);
  v[4] = csub(r1, i1);
  v[2] = cadd(r2, i2);
  v[3] = csub(r2, i2);
}

// Stockham FFT of Wt columns of length L held in LDS (row-major [L][Wt]).
// Returns the buffer that holds the result.
__device__ float2* fft_lds(float2* b0, float2* b1, const float2* tw, int L, int Wt,
                           int dir, const int* rad, int nrad) {
  int Ns = 1;
  for (int s = 0; s < nrad; ++s) {
    const int R = rad[s];
    const int nbf = L / R;
    const int tstep = L / (Ns * R);
    const int total = nbf * Wt;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int col = idx % Wt;
      const int j = idx / Wt;
      const int k = j % Ns;
      float2 v[5];
#pragma unroll
      for (int r = 0; r < 5; ++r)
        if (r < R) v[r] = b0[(j + r * nbf) * Wt + col];
#pragma unroll
      for (int r = 1; r < 5; ++r) {
        if (r < R) {
          float2 w = tw[k * r * tstep];
          if (dir > 0) w.y = -w.y;
          v[r] = cmul(v[r], w);
        }
      }
      switch (R) {
        case 2: dft2(v); break;
        case 3: dft3(v, dir); break;
        case 4: dft4(v, dir); break;
        default: dft5(v, dir); break;
      }
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < 5; ++r)
        if (r < R) b1[(base + r * Ns) * Wt + col] = v[r];
    }
    __syncthreads();
    float2* t = b0;
    b0 = b1;
    b1 = t;
    Ns *= R;
  }
  return b0;
}

__device__ __forceinline__ int wrap_row(int t, int n, int L) {
  int r = t - n / 2;
  return r < 0 ? r + L : r;
}

__global__ __launch_bounds__(256) void k_axis_pass(PassArgs a) {
  extern __shared__ float2 smem[];
  const int L = a.L, Wt = a.Wt;
  float2* b0 = smem;
  float2* b1 = smem + (size_t)L * Wt;
  float2* tw = smem + (size_t)2 * L * Wt;
  __shared__ int rad[kMaxRadices];
  const long long blk = blockIdx.x;
  const long long outer = blk / a.nblk;
  const long long col0 = (blk - outer * a.nblk) * Wt;
  const int ncol = (int)min((long long)Wt, a.inner - col0);
  const int tid = threadIdx.x, bd = blockDim.x;

  if (tid < kMaxRadices) rad[tid] = a.rad[tid];
  for (int i = tid; i < L; i += bd) tw[i] = a.tw[i];
  if (a.n_in < L || ncol < Wt)
    for (int i = tid; i < L * Wt; i += bd) b0[i] = make_float2(0.f, 0.f);
  __syncthreads();

  // ---- load ---------------------------------------------------------------
  for (int idx = tid; idx < a.n_in * Wt; idx += bd) {
    const int t = idx / Wt, col = idx % Wt;
    if (col >= ncol) continue;
    const long long ci = col0 + col;
    const long long p = ci / a.cb;
    const int c = (int)(ci - p * a.cb);
    float2 v;
    if (a.prologue == PRO_IMAGE) {
      const long long pix = (long long)t * a.P + p;
      const float2 xv = a.img[pix];
      const float2 m = a.maps[pix * a.maps_ldc + a.maps_c0 + c];
      v = cscale(cmul(xv, m), a.da[t] * a.dp[p]);
    } else {
      v = a.src[outer * a.src_os + (long long)t * a.src_rs + p * a.src_ldc + a.src_c0 + c];
    }
    if (a.premask && a.mask[outer * a.mask_os + (long long)t * a.mask_rs] == 0)
      v = make_float2(0.f, 0.f);
    const int row = a.pad_in ? wrap_row(t, a.n_in, L) : t;
    b0[row * Wt + col] = v;
  }
  __syncthreads();

  float2* r = fft_lds(b0, b1, tw, L, Wt, a.dir, rad, a.nrad);

  if (a.mid != MID_NONE) {
    for (int idx = tid; idx < L * Wt; idx += bd) {
      const int row = idx / Wt;
      if (a.mask[outer * a.mask_os + (long long)row * a.mask_rs] == 0)
        r[idx] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    if (a.mid == MID_MASK_IFFT) {
      float2* other = (r == b0) ? b1 : b0;
      r = fft_lds(r, other, tw, L, Wt, -a.dir, rad, a.nrad);
    }
  }

  // ---- store --------------------------------------------------------------
  if (a.epilogue == EPI_IMAGE) {
    const int npix = ncol / a.cb;
    const long long p0 = col0 / a.cb;
    for (int idx = tid; idx < a.n_out * npix; idx += bd) {
      const int t = idx / npix, pl = idx % npix;
      const int row = a.pad_out ? wrap_row(t, a.n_out, L) : t;
      const long long p = p0 + pl;
      const long long pix = (long long)t * a.P + p;
      const float2* mp = a.maps + pix * a.maps_ldc + a.maps_c0;
      const float2* rv = r + row * Wt + pl * a.cb;
      float2 acc = make_float2(0.f, 0.f);
      for (int c = 0; c < a.cb; ++c) acc = cadd(acc, cmulc(mp[c], rv[c]));
      acc = cscale(acc, a.da[t] * a.dp[p]);
      if (a.accumulate) acc = cadd(acc, a.img_out[pix]);
      a.img_out[pix] = acc;
    }
  } else {
    for (int idx = tid; idx < a.n_out * Wt; idx += bd) {
      const int t = idx / Wt, col = idx % Wt;
      if (col >= ncol) continue;
      const int row = a.pad_out ? wrap_row(t, a.n_out, L) : t;
      const long long ci = col0 + col;
      const long long p = ci / a.cb;
      const int c = (int)(ci - p * a.cb);
      a.dst[outer * a.dst_os + (long long)t * a.dst_rs + p * a.dst_ldc + a.dst_c0 + c] =
          r[row * Wt + col];
    }
  }
}

// ---------------------------------------------------------------------------
// Specialised pass for a compile-time length L and column-group width TC:
// thread (tr, tc) owns column tc of the panel and butterflies tr, tr + TR, ...
// of every stage; each stage reads its inputs into registers, synchronises,
// and writes the outputs back in place, so one LDS buffer suffices and all
// index arithmetic of the stages is resolved at compile time.
// ---------------------------------------------------------------------------
struct RadPlan {
  int n;
  int r[kMaxRadices];
};

constexpr RadPlan make_radplan(int L) {
  RadPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  while (L % 4 == 0) { p.r[p.n++] = 4; L /= 4; }
  while (L % 2 == 0) { p.r[p.n++] = 2; L /= 2; }
  while (L % 3 == 0) { p.r[p.n++] = 3; L /= 3; }
  while (L % 5 == 0) { p.r[p.n++] = 5; L /= 5; }
  return p;
}

template <int R>
__device__ __forceinline__ void dftR(float2* v, int dir) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3(v, dir);
  else if constexpr (R == 4) dft4(v, dir);
  else dft5(v, dir);
}

// DIR (-1 forward, +1 inverse) is a template parameter so that the
// multiplications by +-i and the twiddle conjugation fold at compile time
// a column group of TC columns uses TR = 256 / TC rows of threads (NT = TR TC
// threads, 252 for TC = 12)
template <int TC>
constexpr int pass_rows() {
  return 256 / TC;
}

template <int L, int TC, int R, int NS, int DIR>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* tw, int tr, int tc) {
  constexpr int TR = pass_rows<TC>();
  constexpr int NBF = L / R;
  constexpr int NB = (NBF + TR - 1) / TR;
  constexpr int TSTEP = L / (NS * R);
  float2 v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = tr + b * TR;
    if (NB * TR == NBF || j < NBF) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[(j + r * NBF) * TC + tc];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = tr + b * TR;
    if (NB * TR == NBF || j < NBF) {
      const int k = j % NS;
      // the first stage's twiddles are all e^0 = 1 (exactly): skipped
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[k * r * TSTEP];
          if (DIR > 0) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      dftR<R>(v[b], DIR);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * NS) * TC + tc] = v[b][r];
    }
  }
  __syncthreads();
}

template <int L, int TC, int S, int NS, int DIR>
__device__ __forceinline__ void fft_stages(float2* buf, const float2* tw, int tr, int tc) {
  constexpr RadPlan P = make_radplan(L);
  if constexpr (S < P.n) {
    constexpr int R = P.r[S];
    fft_stage<L, TC, R, NS, DIR>(buf, tw, tr, tc);
    fft_stages<L, TC, S + 1, NS * R, DIR>(buf, tw, tr, tc);
  }
}

template <int L, int TC>
__device__ __forceinline__ void fft_panel(float2* buf, const float2* tw, int tr, int tc,
                                          int dir) {
  if (dir < 0)
    fft_stages<L, TC, 0, 1, -1>(buf, tw, tr, tc);
  else
    fft_stages<L, TC, 0, 1, 1>(buf, tw, tr, tc);
}

template <int L, int TC>
__global__ __launch_bounds__(256) void k_pass_t(PassArgs a) {
  constexpr int TR = pass_rows<TC>();
  constexpr int NT = TR * TC;
  extern __shared__ float2 smem[];
  float2* buf = smem;             // [L][TC]
  float2* tw = smem + L * TC;     // [L]
  const int tid = threadIdx.x;
  const int tc = tid % TC, tr = tid / TC;
  // panels next to each other in memory (sharing cache lines) on one L2
  const long long blk = a.xcd ? xcd_contiguous(blockIdx.x, gridDim.x) : (long long)blockIdx.x;
  const long long outer = blk / a.nblk;
  const long long col0 = (blk - outer * a.nblk) * a.Wt;
  const int ncol = (int)min((long long)a.Wt, a.inner - col0);
  const bool colok = tc < ncol;
  const long long ci = col0 + tc;
  const long long p = colok ? ci / a.cb : 0;
  const int c = colok ? (int)(ci - p * a.cb) : 0;

  for (int i = tid; i < L; i += NT) tw[i] = a.tw[i];
  if (a.n_in < L)
    for (int r = tr; r < L; r += TR) buf[r * TC + tc] = make_float2(0.f, 0.f);
  __syncthreads();

  // rows t = tr + i TR, i < NR: a thread's rows are loaded in one unrolled
  // sweep (every load issued before the first wait) and then stored to LDS
  constexpr int NR = (L + TR - 1) / TR;
  // paired columns: thread (rv, tp) moves columns 2 tp, 2 tp + 1 of rows
  // rv + i RV as one 16-byte access
  constexpr int TP = TC / 2, RV = NT / TP, NRV = (L + RV - 1) / RV;
  static_assert(TC % 2 == 0 && NT % TP == 0, "column pairs");
  if (a.vec_in) {
    const int tp = tid % TP, rv = tid / TP;
    if (2 * tp < ncol) {
      const float4* s4 = reinterpret_cast<const float4*>(a.src + outer * a.src_os + col0) + tp;
      const long long rs4 = a.src_rs / 2;
      float4 w[NRV];
#pragma unroll
      for (int i = 0; i < NRV; ++i) {
        const int t = rv + i * RV;
        w[i] = t < a.n_in ? s4[(long long)t * rs4] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < NRV; ++i) {
        const int t = rv + i * RV;
        if (t < a.n_in)
          *reinterpret_cast<float4*>(buf + (a.pad_in ? wrap_row(t, a.n_in, L) : t) * TC +
                                     2 * tp) = w[i];
      }
    }
  } else if (a.vec_img) {
    // image prologue on column pairs: both columns are coils of one pixel
    // (even cb), whose map values are adjacent
    const int tp = tid % TP, rv = tid / TP;
    if (2 * tp < ncol) {
      const long long ci2 = col0 + 2 * tp;
      const long long pp = ci2 / a.cb;
      const int cc = (int)(ci2 - pp * a.cb);
      const float dpv = a.dp[pp];
      float4 w[NRV];
#pragma unroll
      for (int i = 0; i < NRV; ++i) {
        const int t = rv + i * RV;
        w[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t < a.n_in) {
          const long long pix = (long long)t * a.P + pp;
          const float2 xv = a.img[pix];
          const float4 m =
              *reinterpret_cast<const float4*>(a.maps + pix * a.maps_ldc + a.maps_c0 + cc);
          const float sc = a.da[t] * dpv;
          const float2 v0 = cscale(cmul(xv, make_float2(m.x, m.y)), sc);
          const float2 v1 = cscale(cmul(xv, make_float2(m.z, m.w)), sc);
          w[i] = make_float4(v0.x, v0.y, v1.x, v1.y);
        }
      }
#pragma unroll
      for (int i = 0; i < NRV; ++i) {
        const int t = rv + i * RV;
        if (t < a.n_in)
          *reinterpret_cast<float4*>(buf + (a.pad_in ? wrap_row(t, a.n_in, L) : t) * TC +
                                     2 * tp) = w[i];
      }
    }
  } else if (colok) {
    const uint8_t* mrow = a.premask ? a.mask + outer * a.mask_os : nullptr;
    float2 v[NR];
    if (a.prologue == PRO_IMAGE) {
      const float dpv = a.dp[p];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        v[i] = make_float2(0.f, 0.f);
        if (t < a.n_in) {
          const long long pix = (long long)t * a.P + p;
          v[i] = cscale(cmul(a.img[pix], a.maps[pix * a.maps_ldc + a.maps_c0 + c]),
                        a.da[t] * dpv);
        }
      }
    } else {
      const float2* src = a.src + outer * a.src_os + p * a.src_ldc + a.src_c0 + c;
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        v[i] = t < a.n_in ? src[(long long)t * a.src_rs] : make_float2(0.f, 0.f);
      }
    }
    if (mrow) {
      // the mask bytes of all rows, then the zeroing (no load waits between)
      uint8_t mk[NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        mk[i] = t < a.n_in ? mrow[(long long)t * a.mask_rs] : (uint8_t)1;
      }
#pragma unroll
      for (int i = 0; i < NR; ++i)
        if (mk[i] == 0) v[i] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int t = tr + i * TR;
      if (t < a.n_in) buf[(a.pad_in ? wrap_row(t, a.n_in, L) : t) * TC + tc] = v[i];
    }
  }
  __syncthreads();

  fft_panel<L, TC>(buf, tw, tr, tc, a.dir);

  if (a.mid != MID_NONE) {
    const uint8_t* mrow = a.mask + outer * a.mask_os;
    for (int r = tr; r < L; r += TR)
      if (mrow[(long long)r * a.mask_rs] == 0) buf[r * TC + tc] = make_float2(0.f, 0.f);
    __syncthreads();
    if (a.mid == MID_MASK_IFFT) fft_panel<L, TC>(buf, tw, tr, tc, -a.dir);
  }

  if (a.epilogue == EPI_IMAGE) {
    // every (pixel, coil) thread forms conj(c_j) times its rows' values in
    // place (map loads of all rows issued together), then the pixel's first
    // thread sums its coils in order
    if (colok) {
      float2 m[NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        m[i] = make_float2(0.f, 0.f);
        if (t < a.n_out) m[i] = a.maps[((long long)t * a.P + p) * a.maps_ldc + a.maps_c0 + c];
      }
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        if (t < a.n_out) {
          float2* rv = buf + (a.pad_out ? wrap_row(t, a.n_out, L) : t) * TC + tc;
          *rv = cmulc(m[i], *rv);
        }
      }
    }
    __syncthreads();
    if (a.sum_rows) {
      // the coil sums spread over all threads, one (row, pixel) each, every
      // pixel's coils still added in order
      const int npix = ncol / a.cb;
      const long long p0 = col0 / a.cb;
      for (int k = tid; k < npix * a.n_out; k += NT) {
        const int t = k / npix, j = k - t * npix;
        const long long pp = p0 + j;
        const float2* rv = buf + (a.pad_out ? wrap_row(t, a.n_out, L) : t) * TC + j * a.cb;
        float2 acc = make_float2(0.f, 0.f);
        for (int cc = 0; cc < a.cb; ++cc) acc = cadd(acc, rv[cc]);
        const long long o = (long long)t * a.P + pp;
        a.img_out[o] = cscale_add(acc, a.da[t] * a.dp[pp], a.accumulate,
                                  a.accumulate ? a.img_out[o] : make_float2(0.f, 0.f));
      }
    } else if (colok && c == 0) {
      const float dpv = a.dp[p];
      float2 prev[NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        prev[i] = a.accumulate && t < a.n_out ? a.img_out[(long long)t * a.P + p]
                                              : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int t = tr + i * TR;
        if (t < a.n_out) {
          const float2* rv = buf + (a.pad_out ? wrap_row(t, a.n_out, L) : t) * TC + tc;
          float2 acc = make_float2(0.f, 0.f);
          for (int cc = 0; cc < a.cb; ++cc) acc = cadd(acc, rv[cc]);
          a.img_out[(long long)t * a.P + p] = cscale_add(acc, a.da[t] * dpv, a.accumulate, prev[i]);
        }
      }
    }
  } else if (a.vec_out) {
    const int tp = tid % TP, rv = tid / TP;
    if (2 * tp < ncol) {
      float4* d4 = reinterpret_cast<float4*>(a.dst + outer * a.dst_os + col0) + tp;
      const long long rs4 = a.dst_rs / 2;
      for (int t = rv; t < a.n_out; t += RV) {
        const int row = a.pad_out ? wrap_row(t, a.n_out, L) : t;
        d4[(long long)t * rs4] = *reinterpret_cast<const float4*>(buf + row * TC + 2 * tp);
      }
    }
  } else if (colok) {
    float2* dst = a.dst + outer * a.dst_os + p * a.dst_ldc + a.dst_c0 + c;
    for (int t = tr; t < a.n_out; t += TR) {
      const int row = a.pad_out ? wrap_row(t, a.n_out, L) : t;
      dst[(long long)t * a.dst_rs] = buf[row * TC + tc];
    }
  }
}

using PassKernel = void (*)(PassArgs);

// column-group widths with a kernel: 12 and 24 / 48 fit 12-coil panels
// (one, two or four pixels), 16 / 32 / 64 the powers of two
constexpr int kPassTC[6] = {12, 16, 24, 32, 48, 64};

int pass_tc_for(int w) {
  for (int tc : kPassTC)
    if (w <= tc) return tc;
  return 0;
}

template <int L>
PassKernel pick_tc(int TC) {
  switch (TC) {
    case 12: return k_pass_t<L, 12>;
    case 16: return k_pass_t<L, 16>;
    case 24: return k_pass_t<L, 24>;
    case 32: return k_pass_t<L, 32>;
    case 48: return k_pass_t<L, 48>;
    case 64: return k_pass_t<L, 64>;
    default: return nullptr;
  }
}

PassKernel specialised(int L, int TC) {
  switch (L) {
    case 20: return pick_tc<20>(TC);
    case 30: return pick_tc<30>(TC);
    case 40: return pick_tc<40>(TC);
    case 48: return pick_tc<48>(TC);
    case 60: return pick_tc<60>(TC);
    case 64: return pick_tc<64>(TC);
    case 80: return pick_tc<80>(TC);
    case 96: return pick_tc<96>(TC);
    case 120: return pick_tc<120>(TC);
    case 128: return pick_tc<128>(TC);
    case 160: return pick_tc<160>(TC);
    case 192: return pick_tc<192>(TC);
    case 240: return pick_tc<240>(TC);
    case 256: return pick_tc<256>(TC);
    case 320: return pick_tc<320>(TC);
    case 384: return pick_tc<384>(TC);
    case 480: return pick_tc<480>(TC);
    default: return nullptr;
  }
}

bool factorize(int L, int* rad, int* nrad) {
  int n = L, k = 0;
  while (n % 4 == 0 && k < kMaxRadices) { rad[k++] = 4; n /= 4; }
  while (n % 2 == 0 && k < kMaxRadices) { rad[k++] = 2; n /= 2; }
  while (n % 3 == 0 && k < kMaxRadices) { rad[k++] = 3; n /= 3; }
  while (n % 5 == 0 && k < kMaxRadices) { rad[k++] = 5; n /= 5; }
  *nrad = k;
  return n == 1;
}

}  // namespace

int get_plan(cs_ctx* c, int L, const FFTPlan** out) {
  auto it = c->plans.find(L);
  if (it != c->plans.end()) {
    *out = &it->second;
    return CS_OK;
  }
  if (L < 1 || L > kMaxFFT)
    return fail(c, CS_EINVAL, "FFT length " + std::to_string(L) + " out of range");
  FFTPlan p;
  p.L = L;
  if (!factorize(L, p.rad, &p.nrad))
    return fail(c, CS_EINVAL, "FFT length " + std::to_string(L) +
                                  " has a prime factor other than 2, 3, 5");
  std::vector<float2> tw(L);
  for (int k = 0; k < L; ++k) {
    const double ang = -2.0 * M_PI * (double)k / (double)L;
    tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  CS_HIP(c, hipMalloc(&p.tw, sizeof(float2) * L));
  CS_HIP(c, hipMemcpy(p.tw, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice));
  c->plans[L] = p;
  *out = &c->plans[L];
  return CS_OK;
}

void fill_plan(PassArgs& a, const FFTPlan* p) {
  a.L = p->L;
  a.nrad = p->nrad;
  for (int i = 0; i < kMaxRadices; ++i) a.rad[i] = p->rad[i];
  a.tw = p->tw;
}

int launch_pass(cs_ctx* c, PassArgs& a, long long n_outer) {
  const int L = a.L;
  const bool image_cols = (a.prologue == PRO_IMAGE || a.epilogue == EPI_IMAGE);
  if (a.n_in > L || a.n_out > L) return fail(c, CS_EINVAL, "pass rows exceed FFT length");
  if (image_cols && (a.inner % a.cb) != 0)
    return fail(c, CS_EINVAL, "image pass columns not a multiple of the coil count");
  if (specialised(L, 16) != nullptr && a.cb <= 64) {
    // panel width: image passes take whole pixels (c->fft_pix of them, all
    // coils of each), grid passes c->fft_cols columns; the column group is
    // the narrowest kernel width that holds the panel, kept to at most 40
    // elements per thread (registers) and a 96 KiB LDS buffer
    // (only the coil-sum epilogue needs all coils of a pixel in one panel; an
    // image prologue alone works per column, and with c->fft_pro_cols > 0
    // takes panels of that many columns)
    const bool whole_pix = a.epilogue == EPI_IMAGE || (image_cols && c->fft_pro_cols <= 0);
    long long w = whole_pix ? (long long)a.cb * std::max(1, c->fft_pix)
                            : (image_cols ? c->fft_pro_cols : c->fft_cols);
    if (w > a.inner) w = a.inner;
    auto fits = [&](int tc) {
      return tc > 0 && (long long)L * tc <= 40LL * 256 &&
             sizeof(float2) * ((size_t)L * tc + L) <= 96 * 1024;
    };
    int TC = pass_tc_for((int)w);
    while (!fits(TC) && w > (whole_pix ? a.cb : 1)) {
      w = whole_pix ? std::max<long long>(a.cb, w - a.cb) : std::max<long long>(1, w / 2);
      TC = pass_tc_for((int)w);
    }
    if (fits(TC)) {
      a.xcd = c->fft_xcd;
      a.Wt = (int)w;
      // column pairs: contiguous columns (ldc = cb, c0 = 0), every row and
      // panel start on an even column and 16-byte aligned pointers
      const bool even = a.Wt % 2 == 0 && a.inner % 2 == 0;
      a.vec_in = c->fft_vec && even && a.prologue == PRO_GRID && !a.premask &&
                 a.src_ldc == a.cb && a.src_c0 == 0 && a.src_os % 2 == 0 &&
                 a.src_rs % 2 == 0 && ((uintptr_t)a.src & 15) == 0;
      a.vec_out = c->fft_vec && even && a.epilogue != EPI_IMAGE && a.dst_ldc == a.cb &&
                  a.dst_c0 == 0 && a.dst_os % 2 == 0 && a.dst_rs % 2 == 0 &&
                  ((uintptr_t)a.dst & 15) == 0;
      a.sum_rows = c->fft_sum_rows;
      // image prologue on coil pairs of one pixel (even cb and map offsets)
      a.vec_img = c->fft_vec_img && even && a.prologue == PRO_IMAGE && !a.premask &&
                  a.cb % 2 == 0 && a.maps_ldc % 2 == 0 && a.maps_c0 % 2 == 0 &&
                  ((uintptr_t)a.maps & 15) == 0;
      const long long nblk = (a.inner + a.Wt - 1) / a.Wt;
      a.nblk = nblk;
      if (nblk * n_outer > 0x7fffffffLL || n_outer < 1)
        return fail(c, CS_EINVAL, "pass grid too large");
      const size_t lds = sizeof(float2) * ((size_t)L * TC + L);
      PassKernel k = specialised(L, TC);
      if (lds > 64 * 1024)
        CS_HIP(c, hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
      const int nt = (256 / TC) * TC;
      CS_KLAUNCH(c, K_PASS, k, dim3((unsigned)(nblk * n_outer)), dim3(nt), lds, c->stream, a);
      CS_HIP(c, hipGetLastError());
      return CS_OK;
    }
  }
  // panel width: as many columns as fit a 64 KiB LDS budget, a multiple of
  // cb when the columns are (pixel, coil) pairs of an image pass
  const long long budget = 64 * 1024 / sizeof(float2);
  long long w = (budget - L) / (2LL * L);
  if (image_cols) w = (w / a.cb) * a.cb;
  if (w < (image_cols ? a.cb : 1)) w = image_cols ? a.cb : 1;
  if (w > a.inner) w = a.inner;
  if (image_cols && (a.inner % a.cb) != 0)
    return fail(c, CS_EINVAL, "image pass columns not a multiple of the coil count");
  a.Wt = (int)w;
  const size_t lds = sizeof(float2) * ((size_t)2 * L * a.Wt + L);
  if (lds > 160 * 1024)
    return fail(c, CS_EINVAL, "FFT panel does not fit in LDS");
  if (a.n_in > L || a.n_out > L)
    return fail(c, CS_EINVAL, "pass rows exceed FFT length");
  const long long nblk = (a.inner + a.Wt - 1) / a.Wt;
  a.nblk = nblk;
  if (nblk * n_outer > 0x7fffffffLL || n_outer < 1)
    return fail(c, CS_EINVAL, "pass grid too large");
  dim3 grid((unsigned)(nblk * n_outer));
  if (lds > 64 * 1024)
    CS_HIP(c, hipFuncSetAttribute((const void*)k_axis_pass,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  CS_KLAUNCH(c, K_PASS, k_axis_pass, grid, dim3(256), lds, c->stream, a);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

}  // namespace cs
