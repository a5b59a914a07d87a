// Kaiser-Bessel gridding for the non-uniform FFT of Sec. 2.1 (F~ = F~_n,
// implemented as a NUFFT after Beatty et al. 2005) with density compensation
// A = W^1/2 F C (Sec. 2.1.1).
//
// Set-up (once per operator, host): each sample's grid coordinate
// u_a = k_a m_a / n_a gives its first tap floor(u_a) - 1 and the four
// per-axis kernel weights phi(u_a - g) (FP64, stored as FP32).  Samples are
// sorted by the 8x8x8 (3D) or 16x16 (2D) grid tile that holds their first tap,
// and every tile gets the list of samples whose 4^d footprint reaches it.
//
// interp: one thread per sorted sample gathers the 4^d taps of every coil of
//         a coil chunk (coil-fastest grid, so each tap is one contiguous
//         vector of coils).
// spread: one work-group per output tile accumulates, in LDS, the
//         contributions of the samples on its list that land inside the tile,
//         one sample at a time with one lane per tap.  Within a LDS
//         instruction all lanes address distinct voxels and a wave executes
//         its LDS instructions in order, so the summation order of every voxel
//         is fixed: the result is deterministic and no global atomics are
//         used.  Every voxel of the tile is then written once.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>

#include "cs_internal.h"

namespace cs {

// I0 by its power series sum (x^2/4)^k / (k!)^2 (converges for all x; the
// argument here is at most beta ~ 7).
double kb_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

// Fourier transform of the KB kernel I0(beta sqrt(1 - (2t/W)^2)) on |t| <= W/2
// at frequency nu: W sinh(sqrt(beta^2 - (pi W nu)^2)) / sqrt(...).
double kb_ft(double nu, double W, double beta) {
  const double a = beta * beta - (M_PI * W * nu) * (M_PI * W * nu);
  if (a > 0) {
    const double s = std::sqrt(a);
    return W * std::sinh(s) / s;
  }
  if (a < 0) {
    const double s = std::sqrt(-a);
    return W * std::sin(s) / s;
  }
  return W;
}

namespace {

double kb_kernel(double t, double W, double beta) {
  const double z = 1.0 - (2.0 * t / W) * (2.0 * t / W);
  return z >= 0 ? kb_i0(beta * std::sqrt(z)) : 0.0;
}

template <int NDIM, int CBT>
__global__ __launch_bounds__(256) void k_interp(const float2* __restrict__ G, int mx,
                                                int my, int mz, int cb,
                                                const SampleRec* __restrict__ rec,
                                                long long N, int wmode,
                                                float2* __restrict__ out, int ldc, int c0,
                                                int caller_order) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const SampleRec r = rec[j];
  float2 acc[CBT];
#pragma unroll
  for (int c = 0; c < CBT; ++c) acc[c] = make_float2(0.f, 0.f);
  int xs[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    int v = r.bx + d;
    xs[d] = v >= mx ? v - mx : v;
  }
  const int nzt = NDIM == 3 ? 4 : 1;
  // keep the z / y tap loops rolled: unrolling them lets the compiler hoist
  // all 64 taps' loads and spill
#pragma unroll 1
  for (int dz = 0; dz < nzt; ++dz) {
    int z = r.bz + dz;
    if (z >= mz) z -= mz;
    const float wz = NDIM == 3 ? r.wz[dz] : 1.f;
#pragma unroll 1
    for (int dy = 0; dy < 4; ++dy) {
      int y = r.by + dy;
      if (y >= my) y -= my;
      const float wyz = wz * r.wy[dy];
      const long long row = ((long long)z * my + y) * mx;
#pragma unroll
      for (int dx = 0; dx < 4; ++dx) {
        const float w = wyz * r.wx[dx];
        const float2* p = G + (row + xs[dx]) * cb;
        if constexpr (CBT % 2 == 0) {
          // cb == CBT (even): two coils per 16-byte load
          const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
          for (int c = 0; c < CBT / 2; ++c) {
            const float4 g = p4[c];
            acc[2 * c].x += w * g.x;
            acc[2 * c].y += w * g.y;
            acc[2 * c + 1].x += w * g.z;
            acc[2 * c + 1].y += w * g.w;
          }
        } else {
#pragma unroll
          for (int c = 0; c < CBT; ++c) {
            if (c < cb) {
              const float2 g = p[c];
              acc[c].x += w * g.x;
              acc[c].y += w * g.y;
            }
          }
        }
      }
    }
  }
  const float s = wmode == W_FULL ? r.w : (wmode == W_SQRT ? r.sw : 1.f);
  const long long o = caller_order ? (long long)r.orig : j;
  float2* dst = out + o * ldc + c0;
#pragma unroll
  for (int c = 0; c < CBT; ++c)
    if (c < cb) dst[c] = make_float2(acc[c].x * s, acc[c].y * s);
}

__device__ __forceinline__ float sel4(const float* w, int i) {
  return i == 0 ? w[0] : (i == 1 ? w[1] : (i == 2 ? w[2] : w[3]));
}

// Tile geometry of the spread: 8x8xTZ3 (3D, TZ3 = 4 or 8) or 16x16 (2D)
// voxels.  The LDS accumulator is planar per (coil, re/im) with voxel offset
// lz * PZ + ly * PY + lx; PY = 8, PZ = 68 (3D) and PY = 20 (2D) make the 32
// lanes of each half-wave (one lane per tap) hit 32 distinct banks.
template <int NDIM, int TZ3>
struct SpreadTile {
  static constexpr int TX = NDIM == 3 ? 8 : 16;
  static constexpr int TY = NDIM == 3 ? 8 : 16;
  static constexpr int TZ = NDIM == 3 ? TZ3 : 1;
  static constexpr int PY = NDIM == 3 ? 8 : 20;
  static constexpr int PZ = NDIM == 3 ? 68 : 0;
  static constexpr int PLANE = NDIM == 3 ? TZ * PZ : TY * PY;
  static constexpr int NVOX = TX * TY * TZ;
};

constexpr int kSpreadBatch = 64;   // samples staged in LDS per step

// One work item = one output tile and a contiguous chunk of its sample list
// (samples whose footprint reaches the tile, in sorted order).  Lane l of
// each wave owns tap (l & 3, (l >> 2) & 3, l >> 4) of the current sample.
// Consecutive samples with the same first tap touch the same voxels, so a
// lane accumulates such a run in registers and adds the run's sum into the
// LDS tile once (one ds_add per coil and part; the lanes of one instruction
// address distinct voxels, and a wave issues its LDS operations in order, so
// every voxel's summation order is fixed).  Items that cover a whole tile
// write it to the grid; items of a split tile write a partial tile that the
// merge kernel sums in item order.
template <int NDIM, int TZ3, int NW, int CBW>
__global__ __launch_bounds__(64 * NW) void k_spread(
    const float2* __restrict__ V, int cb, const SampleRec* __restrict__ rec,
    const int4* __restrict__ items, const int* __restrict__ tile_list, int ntx, int nty,
    int mx, int my, int mz, float2* __restrict__ G, float2* __restrict__ partial) {
  using T = SpreadTile<NDIM, TZ3>;
  constexpr int NT = 64 * NW;  // NW waves, each owning a contiguous share of the coils
  extern __shared__ float lds[];
  constexpr int SRP = 17;  // staged record pitch (odd: conflict-free writes)
  float* acc = lds;                                   // [cb][2][PLANE]
  float* srec = lds + (size_t)cb * 2 * T::PLANE;      // [batch][SRP]
  float2* sv = reinterpret_cast<float2*>(srec + kSpreadBatch * SRP + 1);  // [batch][NW CBW]

  const int4 it = items[blockIdx.x];
  const int tile = it.x, kbeg = it.y, kend = it.z, slot = it.w;
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int x0 = ix * T::TX, y0 = iy * T::TY, z0 = iz * T::TZ;
  const int ex = min(T::TX, mx - x0), ey = min(T::TY, my - y0), ez = min(T::TZ, mz - z0);
  const int tid = threadIdx.x;
  for (int i = tid; i < cb * 2 * T::PLANE; i += NT) acc[i] = 0.f;

  const int wave = tid >> 6, lane = tid & 63;
  const int cbw = (cb + NW - 1) / NW;
  const int c_lo = wave * cbw;
  const int c_n = max(0, min(cb, c_lo + cbw) - c_lo);
  const int dx = lane & 3, dy = (lane >> 2) & 3, dz = lane >> 4;
  const bool lane_ok = NDIM == 3 || dz == 0;

  float2 racc[CBW];
#pragma unroll
  for (int q = 0; q < CBW; ++q) racc[q] = make_float2(0.f, 0.f);
  int rbx = -1, rby = -1, rbz = -1;
  int raddr = 0;
  bool rin = false;

  __shared__ int s_rs[kSpreadBatch];  // run starts of the staged batch
  __shared__ int s_nr;
  constexpr int pitch = NW * CBW;     // staged value row; each wave reads CBW slots

  // Staging is double-buffered through registers: the loads of batch b + 1
  // are issued before batch b is processed.  Thread t < 64 fetches sample t's
  // record; thread t fetches coil share (t % NW) of sample t / NW.
  int pb[3] = {0, 0, 0};
  float pw[12];
  float2 pv[CBW];
  const int vs = tid / NW, vh = tid % NW;
  auto prefetch = [&](int k0, int n) {
    if (tid < n) {
      const SampleRec& r = rec[tile_list[k0 + tid]];
      pb[0] = r.bx; pb[1] = r.by; pb[2] = r.bz;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pw[q] = r.wx[q];
        pw[4 + q] = r.wy[q];
        pw[8 + q] = r.wz[q];
      }
    }
    if (vs < n) {
      const float2* src = V + (long long)tile_list[k0 + vs] * cb + vh * cbw;
      const int lim = cb - vh * cbw;
#pragma unroll
      for (int q = 0; q < CBW; ++q)
        if (q < lim && q < cbw) pv[q] = src[q];
    }
  };
  if (kbeg < kend) prefetch(kbeg, min(kSpreadBatch, kend - kbeg));

  for (int k0 = kbeg; k0 < kend; k0 += kSpreadBatch) {
    const int n = min(kSpreadBatch, kend - k0);
    __syncthreads();  // previous batch consumed (and accumulator zeroed)
    if (tid < n) {
      float* d = srec + tid * SRP;
      d[0] = __int_as_float(pb[0]);
      d[1] = __int_as_float(pb[1]);
      d[2] = __int_as_float(pb[2]);
#pragma unroll
      for (int q = 0; q < 12; ++q) d[4 + q] = pw[q];
    }
    if (vs < n) {
      // each thread writes only its own cbw columns (the halves must not overlap)
      float2* dst = sv + vs * pitch + vh * cbw;
#pragma unroll
      for (int q = 0; q < CBW; ++q)
        if (q < cbw) dst[q] = pv[q];
    }
    // run starts: sample s opens a run when its first tap differs from the
    // previous sample's (or from the run carried over from the last batch)
    if (tid < 64) {
      const int qx = __shfl_up(pb[0], 1), qy = __shfl_up(pb[1], 1), qz = __shfl_up(pb[2], 1);
      const int pbx = tid > 0 ? qx : rbx, pby = tid > 0 ? qy : rby, pbz = tid > 0 ? qz : rbz;
      const bool start = tid < n && (pb[0] != pbx || pb[1] != pby || pb[2] != pbz);
      const unsigned long long mask = __ballot(start);
      if (start) s_rs[__popcll(mask & ((1ull << tid) - 1ull))] = tid;
      if (tid == 0) s_nr = __popcll(mask);
    }
    __syncthreads();
    if (k0 + kSpreadBatch < kend)
      prefetch(k0 + kSpreadBatch, min(kSpreadBatch, kend - k0 - kSpreadBatch));
    const int nr = s_nr;
    int s = 0;
    for (int r = -1; r < nr; ++r) {
      const int s1 = (r + 1 < nr) ? s_rs[r + 1] : n;
      if (r >= 0) {
        // close the current run, open the one starting at s
        if (rin) {
#pragma unroll
          for (int q = 0; q < CBW; ++q) {
            if (q < c_n) {
              float* pl = acc + (size_t)(c_lo + q) * 2 * T::PLANE + raddr;
              atomicAdd(pl, racc[q].x);
              atomicAdd(pl + T::PLANE, racc[q].y);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < CBW; ++q) racc[q] = make_float2(0.f, 0.f);
        const float* d = srec + s * SRP;
        rbx = __float_as_int(d[0]); rby = __float_as_int(d[1]); rbz = __float_as_int(d[2]);
        int gx = rbx + dx;
        if (gx >= mx) gx -= mx;
        int gy = rby + dy;
        if (gy >= my) gy -= my;
        int gz = NDIM == 3 ? rbz + dz : 0;
        if (gz >= mz) gz -= mz;
        const int lx = gx - x0, ly = gy - y0, lz = gz - z0;
        rin = lane_ok && (unsigned)lx < (unsigned)ex && (unsigned)ly < (unsigned)ey &&
              (unsigned)lz < (unsigned)ez;
        raddr = lz * T::PZ + ly * T::PY + lx;
      }
      // samples of the run: register accumulation, no branches
#pragma unroll 2
      for (; s < s1; ++s) {
        const float* d = srec + s * SRP;
        float w = d[4 + dx] * d[8 + dy];
        if (NDIM == 3) w *= d[12 + dz];
        const float2* v = sv + s * pitch + c_lo;
#pragma unroll
        for (int q = 0; q < CBW; ++q) {
          const float2 val = v[q];
          racc[q].x += w * val.x;
          racc[q].y += w * val.y;
        }
      }
    }
  }
  if (rin) {
#pragma unroll
    for (int q = 0; q < CBW; ++q) {
      if (q < c_n) {
        float* pl = acc + (size_t)(c_lo + q) * 2 * T::PLANE + raddr;
        atomicAdd(pl, racc[q].x);
        atomicAdd(pl + T::PLANE, racc[q].y);
      }
    }
  }
  __syncthreads();
  // write-out: element i = voxel v (tile order) * cb + coil; the quotient
  // i / cb (i < 2^13, cb <= 16) is exact in float with the half offset
  const float inv_cb = 1.0f / (float)cb;
  for (int i = tid; i < T::NVOX * cb; i += NT) {
    const int v = (int)(((float)i + 0.5f) * inv_cb);
    const int c = i - v * cb;
    const int lx = v % T::TX, ly = (v / T::TX) % T::TY, lz = v / (T::TX * T::TY);
    if (lx >= ex || ly >= ey || lz >= ez) continue;
    const int e = lz * T::PZ + ly * T::PY + lx;
    const float2 val = make_float2(acc[(size_t)c * 2 * T::PLANE + e],
                                   acc[(size_t)c * 2 * T::PLANE + T::PLANE + e]);
    if (slot < 0) {
      G[(((long long)(z0 + lz) * my + (y0 + ly)) * mx + (x0 + lx)) * cb + c] = val;
    } else {
      const int tv = (lz * T::TY + ly) * T::TX + lx;
      partial[((long long)slot * T::NVOX + tv) * cb + c] = val;
    }
  }
}

// Sum the partial tiles of split tiles in item order.  merges[i] =
// (tile, first slot, slot count, 0).
template <int NDIM, int TZ3>
__global__ void k_spread_merge(const int4* __restrict__ merges, const float2* __restrict__ partial,
                               int cb, int ntx, int nty, int mx, int my, int mz,
                               float2* __restrict__ G) {
  using T = SpreadTile<NDIM, TZ3>;
  // block b handles elements [part * 256, part * 256 + 256) of merge b / nparts
  const int nparts = (T::NVOX * cb + 255) / 256;
  const int4 m = merges[blockIdx.x / nparts];
  const int part = blockIdx.x % nparts;
  const int tile = m.x;
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int x0 = ix * T::TX, y0 = iy * T::TY, z0 = iz * T::TZ;
  const int ex = min(T::TX, mx - x0), ey = min(T::TY, my - y0), ez = min(T::TZ, mz - z0);
  const int i = part * 256 + threadIdx.x;
  if (i >= T::NVOX * cb) return;
  const int v = (int)(((float)i + 0.5f) / (float)cb);  // exact for i < 2^13
  const int c = i - v * cb;
  const int lx = v % T::TX, ly = (v / T::TX) % T::TY, lz = v / (T::TX * T::TY);
  if (lx >= ex || ly >= ey || lz >= ez) return;
  const int tv = v;
  const float2* p = partial + ((long long)m.y * T::NVOX + tv) * cb + c;
  const long long step = (long long)T::NVOX * cb;
  float2 s = make_float2(0.f, 0.f);
#pragma unroll 8
  for (int q = 0; q < m.z; ++q) {
    const float2 pv = p[q * step];
    s.x += pv.x;
    s.y += pv.y;
  }
  G[(((long long)(z0 + lz) * my + (y0 + ly)) * mx + (x0 + lx)) * cb + c] = s;
}

__global__ void k_gather_samples(const float2* __restrict__ y, int ldc, int c0, int cb,
                                 const SampleRec* __restrict__ rec, long long N,
                                 float2* __restrict__ vals) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * cb) return;
  const long long j = i / cb;
  const int c = (int)(i - j * cb);
  const SampleRec& r = rec[j];
  const float2 v = y[(long long)r.orig * ldc + c0 + c];
  vals[i] = make_float2(v.x * r.sw, v.y * r.sw);
}

template <int NDIM>
int interp_dispatch(cs_ctx* c, const float2* grid, int cb, int wmode, float2* out,
                    int ldc, int c0, int caller_order) {
  const long long N = c->N;
  const int bs = 256;
  const unsigned nb = (unsigned)((N + bs - 1) / bs);
#define CS_INTERP(CBT)                                                                \
  CS_KLAUNCH(c, K_INTERP, (k_interp<NDIM, CBT>), dim3(nb), dim3(bs), 0, c->stream, grid,   \
                     c->mx, c->my, c->mz, cb, c->rec, N, wmode, out, ldc, c0,         \
                     caller_order)
  // even chunk sizes get an exact instantiation (vector loads); odd ones use
  // the next odd bound with a runtime guard
  switch (cb) {
    case 2: CS_INTERP(2); break;
    case 4: CS_INTERP(4); break;
    case 6: CS_INTERP(6); break;
    case 8: CS_INTERP(8); break;
    case 10: CS_INTERP(10); break;
    case 12: CS_INTERP(12); break;
    case 14: CS_INTERP(14); break;
    case 16: CS_INTERP(16); break;
    default:
      if (cb <= 3) CS_INTERP(3);
      else if (cb <= 7) CS_INTERP(7);
      else if (cb <= 11) CS_INTERP(11);
      else CS_INTERP(15);
  }
#undef CS_INTERP
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

}  // namespace

int launch_interp(cs_ctx* c, const float2* grid, int cb, int wmode, float2* out,
                  int ldc, int c0, int caller_order) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "interp coil chunk");
  if (c->N == 0) return CS_OK;
  return c->ndim == 3 ? interp_dispatch<3>(c, grid, cb, wmode, out, ldc, c0, caller_order)
                      : interp_dispatch<2>(c, grid, cb, wmode, out, ldc, c0, caller_order);
}

namespace {
template <int NDIM, int TZ3, int NW, int CBW>
int spread_launch(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  using T = SpreadTile<NDIM, TZ3>;
  const size_t lds = sizeof(float) * ((size_t)cb * 2 * T::PLANE + kSpreadBatch * 17 + 1) +
                     sizeof(float2) * (size_t)kSpreadBatch * NW * CBW;
  if (lds > 160 * 1024) return fail(c, CS_EINVAL, "spread tile does not fit in LDS");
  auto kern = k_spread<NDIM, TZ3, NW, CBW>;
  if (lds > 64 * 1024)
    CS_HIP(c, hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
  if (c->n_items > 0)
    CS_KLAUNCH(c, K_SPREAD, kern, dim3((unsigned)c->n_items), dim3(64 * NW), lds, c->stream,
               vals, cb, c->rec, c->items, c->tile_list, c->ntile[2], c->ntile[1], c->mx,
               c->my, c->mz, grid, c->partial);
  CS_HIP(c, hipGetLastError());
  if (c->n_merges > 0) {
    const long long nparts = (T::NVOX * cb + 255) / 256;
    CS_KLAUNCH(c, K_SPREAD, (k_spread_merge<NDIM, TZ3>),
               dim3((unsigned)(c->n_merges * nparts)), dim3(256), 0, c->stream, c->merges,
               c->partial, cb, c->ntile[2], c->ntile[1], c->mx, c->my, c->mz, grid);
  }
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

template <int NDIM, int TZ3, int NW>
int spread_cbw(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  const int cbw = (cb + NW - 1) / NW;  // coils per wave
  if (cbw <= 2) return spread_launch<NDIM, TZ3, NW, 2>(c, vals, cb, grid);
  if (cbw <= 4) return spread_launch<NDIM, TZ3, NW, 4>(c, vals, cb, grid);
  if (cbw <= 6) return spread_launch<NDIM, TZ3, NW, 6>(c, vals, cb, grid);
  if (cbw <= 8 || NW > 1) return spread_launch<NDIM, TZ3, NW, 8>(c, vals, cb, grid);
  if (cbw <= 12) return spread_launch<NDIM, TZ3, 1, 12>(c, vals, cb, grid);
  return spread_launch<NDIM, TZ3, 1, 16>(c, vals, cb, grid);
}

template <int NDIM, int TZ3>
int spread_nw(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  if (c->spread_nw == 1) return spread_cbw<NDIM, TZ3, 1>(c, vals, cb, grid);
  return c->spread_nw == 2 ? spread_cbw<NDIM, TZ3, 2>(c, vals, cb, grid)
                           : spread_cbw<NDIM, TZ3, 4>(c, vals, cb, grid);
}
}  // namespace

int launch_spread(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "spread coil chunk");
  if (c->ndim == 2) return spread_nw<2, 1>(c, vals, cb, grid);
  return c->tile[0] == 4 ? spread_nw<3, 4>(c, vals, cb, grid)
                         : spread_nw<3, 8>(c, vals, cb, grid);
}

int launch_gather_samples(cs_ctx* c, const float2* y, int ldc, int c0, int cb,
                          float2* vals) {
  const long long n = c->N * cb;
  if (n == 0) return CS_OK;
  const int bs = 256;
  CS_KLAUNCH(c, K_GATHER, k_gather_samples, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0,
                     c->stream, y, ldc, c0, cb, c->rec, c->N, vals);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int setup_noncart(cs_ctx* c, const float* coords_dev, const float* dcf_dev) {
  const long long N = c->N;
  const int nd = c->ndim;
  std::vector<float> coords((size_t)N * nd), dcf;
  CS_HIP(c, hipMemcpy(coords.data(), coords_dev, sizeof(float) * N * nd,
                      hipMemcpyDeviceToHost));
  if (dcf_dev) {
    dcf.resize(N);
    CS_HIP(c, hipMemcpy(dcf.data(), dcf_dev, sizeof(float) * N, hipMemcpyDeviceToHost));
    for (long long i = 0; i < N; ++i)
      if (!(dcf[i] >= 0.f)) return fail(c, CS_EINVAL, "density compensation must be >= 0");
  }
  const int n[3] = {c->nz, c->ny, c->nx};
  const int m[3] = {c->mz, c->my, c->mx};
  const double W = 4.0, beta = c->beta;

  // tiles
  if (nd == 3) {
    // tile depth 4 (default) or 8, and waves per spread work-group (2 by
    // default, or 1 or 4) -- the defaults measured fastest on the 3D cones
    // workload:
    // tuning knobs, CS_SPREAD_TZ and CS_SPREAD_NW in the environment
    const char* tz = std::getenv("CS_SPREAD_TZ");
    c->tile[0] = (tz && std::atoi(tz) == 8) ? 8 : 4;
    c->tile[1] = 8;
    c->tile[2] = 8;
    const char* nw = std::getenv("CS_SPREAD_NW");
    const int nwv = nw ? std::atoi(nw) : 2;
    c->spread_nw = (nwv == 1 || nwv == 4) ? nwv : 2;
  } else {
    c->tile[0] = 1; c->tile[1] = 16; c->tile[2] = 16;
  }
  for (int a = 0; a < 3; ++a) c->ntile[a] = (m[a] + c->tile[a] - 1) / c->tile[a];
  c->ntiles = (long long)c->ntile[0] * c->ntile[1] * c->ntile[2];

  std::vector<SampleRec> rec(N);
  std::vector<unsigned long long> key(N);
  for (long long i = 0; i < N; ++i) {
    SampleRec r{};
    int base[3] = {0, 0, 0};
    float* wts[3] = {r.wz, r.wy, r.wx};
    for (int a = 3 - nd; a < 3; ++a) {
      const double k = coords[(size_t)i * nd + (2 - a)];
      if (!(k >= -0.5 * n[a] && k < 0.5 * n[a]))
        return fail(c, CS_EINVAL, "coordinate outside [-n/2, n/2)");
      const double u = k * (double)m[a] / (double)n[a];
      const double f = std::floor(u);
      const long long b = (long long)f - 1;
      for (int j = 0; j < 4; ++j) wts[a][j] = (float)kb_kernel(u - (double)(b + j), W, beta);
      long long bw = b % m[a];
      if (bw < 0) bw += m[a];
      base[a] = (int)bw;
    }
    if (nd == 2) {
      r.wz[0] = 1.f;
      base[0] = 0;
    }
    r.bz = base[0]; r.by = base[1]; r.bx = base[2];
    r.orig = (int)i;
    const double w = dcf_dev ? (double)dcf[i] : 1.0;
    r.w = (float)w;
    r.sw = (float)std::sqrt(w);
    rec[i] = r;
    const long long t = ((long long)(r.bz / c->tile[0]) * c->ntile[1] + r.by / c->tile[1]) *
                            c->ntile[2] + r.bx / c->tile[2];
    const long long vox = ((long long)r.bz * m[1] + r.by) * m[2] + r.bx;
    key[i] = ((unsigned long long)t << 40) | (unsigned long long)vox;
  }
  std::vector<long long> order(N);
  std::iota(order.begin(), order.end(), 0LL);
  std::stable_sort(order.begin(), order.end(),
                   [&](long long a, long long b) { return key[a] < key[b]; });
  std::vector<SampleRec> srec(N);
  for (long long j = 0; j < N; ++j) srec[j] = rec[order[j]];

  // tile lists: every tile reached by a sample's footprint
  std::vector<int> cnt(c->ntiles + 1, 0);
  auto tiles_of = [&](const SampleRec& r, long long* out) -> int {
    int lists[3][2], nl[3];
    const int b[3] = {r.bz, r.by, r.bx};
    for (int a = 0; a < 3; ++a) {
      const int span = (a == 0 && nd == 2) ? 1 : 4;
      nl[a] = 0;
      for (int d = 0; d < span; ++d) {
        int g = b[a] + d;
        if (g >= m[a]) g -= m[a];
        const int ti = g / c->tile[a];
        bool seen = false;
        for (int q = 0; q < nl[a]; ++q) seen |= lists[a][q] == ti;
        if (!seen) lists[a][nl[a]++] = ti;
      }
    }
    int k = 0;
    for (int i0 = 0; i0 < nl[0]; ++i0)
      for (int i1 = 0; i1 < nl[1]; ++i1)
        for (int i2 = 0; i2 < nl[2]; ++i2)
          out[k++] = ((long long)lists[0][i0] * c->ntile[1] + lists[1][i1]) * c->ntile[2] +
                     lists[2][i2];
    return k;
  };
  long long tl[8];
  long long nnz = 0;
  for (long long j = 0; j < N; ++j) {
    const int k = tiles_of(srec[j], tl);
    for (int q = 0; q < k; ++q) cnt[tl[q] + 1]++;
    nnz += k;
  }
  if (nnz > 0x7fffffffLL) return fail(c, CS_EINVAL, "too many samples for tile lists");
  for (long long t = 0; t < c->ntiles; ++t) cnt[t + 1] += cnt[t];
  std::vector<int> fillpos(cnt.begin(), cnt.end() - 1);
  std::vector<int> list(nnz);
  for (long long j = 0; j < N; ++j) {
    const int k = tiles_of(srec[j], tl);
    for (int q = 0; q < k; ++q) list[fillpos[tl[q]]++] = (int)j;
  }

  CS_HIP(c, hipMalloc(&c->rec, sizeof(SampleRec) * std::max(1LL, N)));
  CS_HIP(c, hipMemcpy(c->rec, srec.data(), sizeof(SampleRec) * N, hipMemcpyHostToDevice));
  CS_HIP(c, hipMalloc(&c->tile_off, sizeof(int) * (c->ntiles + 1)));
  CS_HIP(c, hipMemcpy(c->tile_off, cnt.data(), sizeof(int) * (c->ntiles + 1),
                      hipMemcpyHostToDevice));
  CS_HIP(c, hipMalloc(&c->tile_list, sizeof(int) * std::max(1LL, nnz)));
  if (nnz)
    CS_HIP(c, hipMemcpy(c->tile_list, list.data(), sizeof(int) * nnz, hipMemcpyHostToDevice));
  if (dcf_dev) {
    CS_HIP(c, hipMalloc(&c->dcf_orig, sizeof(float) * N));
    CS_HIP(c, hipMemcpy(c->dcf_orig, dcf.data(), sizeof(float) * N, hipMemcpyHostToDevice));
  }

  // spread work items: tiles with long lists are split into chunks whose
  // partial tiles are summed afterwards in chunk order
  const int chunk = 1024;
  std::vector<int4> items, merges;
  int nslots = 0;
  for (long long t = 0; t < c->ntiles; ++t) {
    const int beg = cnt[t], end = cnt[t + 1];
    const int len = end - beg;
    if (len <= chunk) {
      items.push_back(make_int4((int)t, beg, end, -1));
    } else {
      const int n = (len + chunk - 1) / chunk;
      merges.push_back(make_int4((int)t, nslots, n, 0));
      for (int q = 0; q < n; ++q)
        items.push_back(make_int4((int)t, beg + q * chunk, std::min(end, beg + (q + 1) * chunk),
                                  nslots + q));
      nslots += n;
    }
  }
  // heavy items first so that the long lists start early
  std::stable_sort(items.begin(), items.end(),
                   [](const int4& a, const int4& b) { return (a.z - a.y) > (b.z - b.y); });
  c->n_items = (long long)items.size();
  c->n_merges = (long long)merges.size();
  CS_HIP(c, hipMalloc(&c->items, sizeof(int4) * std::max<size_t>(1, items.size())));
  if (!items.empty())
    CS_HIP(c, hipMemcpy(c->items, items.data(), sizeof(int4) * items.size(),
                        hipMemcpyHostToDevice));
  CS_HIP(c, hipMalloc(&c->merges, sizeof(int4) * std::max<size_t>(1, merges.size())));
  if (!merges.empty())
    CS_HIP(c, hipMemcpy(c->merges, merges.data(), sizeof(int4) * merges.size(),
                        hipMemcpyHostToDevice));
  const size_t tvox = (size_t)c->tile[0] * c->tile[1] * c->tile[2];
  CS_HIP(c, hipMalloc(&c->partial,
                      sizeof(float2) * std::max<size_t>(1, (size_t)nslots * tvox * kCoilChunk)));
  return CS_OK;
}

}  // namespace cs
