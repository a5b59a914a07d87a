// Kaiser-Bessel gridding for the non-uniform FFT of Sec. 2.1 (F~ = F~_n,
// implemented as a NUFFT after Beatty et al. 2005) with density compensation
// A = W^1/2 F C (Sec. 2.1.1).
//
// Set-up (once per operator, host): each sample's grid coordinate
// u_a = k_a m_a / n_a gives its first tap floor(u_a) - 1 and the four
// per-axis kernel weights phi(u_a - g) (FP64, stored as FP32).  Samples are
// sorted by the 8x8x8 (3D) or 16x16 (2D) grid tile that holds their first
// tap, then by that tap, and each tile's samples are cut into work items of
// at most 2048 samples.
//
// interp: one thread per sorted sample gathers the 4^d taps of every coil of
//         a coil chunk (coil-fastest grid, so each tap is one contiguous
//         vector of coils).
// spread: one work-group per work item and coil group accumulates, in LDS,
//         its samples into the tile grown by the 3-voxel reach of the kernel
//         (each sample is handled once), one sample at a time with one lane
//         per tap.  Within a LDS instruction all lanes address distinct
//         voxels and a wave executes its LDS instructions in order, so every
//         voxel's summation order is fixed.  The grown tile is written to the
//         item's slot, and a merge kernel sums, for every grid voxel, the
//         slots that cover it in a fixed order: deterministic, and no global
//         atomics.
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

// Halo'd spread tile: every sample belongs to the one tile that holds its
// first tap, and its 4^d footprint stays inside the tile grown by 3 voxels
// along each axis.  The LDS accumulator is planar per (coil, re/im) with
// voxel offset lz * PZ + ly * PY + lx: dense in 3D (the 64 taps of a sample
// meet at most two per bank, and only when a run is flushed) and with row
// pitch 20 in 2D (16 taps in distinct banks).
template <int NDIM>
struct Halo {
  static constexpr int TX = NDIM == 3 ? 8 : 16;
  static constexpr int TY = NDIM == 3 ? 8 : 16;
  static constexpr int TZ = NDIM == 3 ? 8 : 1;
  static constexpr int EX = TX + 3, EY = TY + 3, EZ = NDIM == 3 ? TZ + 3 : 1;
  static constexpr int EXT = EX * EY * EZ;  // voxels of a partial tile
  static constexpr int PY = NDIM == 3 ? EX : 20;
  static constexpr int PZ = NDIM == 3 ? EX * EY : 0;
  static constexpr int PLANE = (EZ - 1) * PZ + (EY - 1) * PY + EX + 1;
  static constexpr int NTAPS = NDIM == 3 ? 64 : 16;
  static constexpr int LPC = 64 / NTAPS;  // coil slots per wave
};

// Tiled interpolation: one work-group per spread work item and coil group.
// The group first copies the item's halo'd tile of the grid (the tile grown
// by the 3-voxel reach of the kernel, wrapped modulo the grid) into LDS,
// planar per (coil, re/im) as in the spreading accumulator, and then one
// thread per sample sums its 4^d taps from LDS in the same order as
// k_interp (z, y, x taps, weight wz wy wx), so both give the same values.
// Every tap of a sample lies in the halo'd tile of the tile that holds its
// first tap, so no other memory is read.
template <int NDIM, int CG, int NT>
__global__ __launch_bounds__(NT) void k_interp_tile(
    const float2* __restrict__ G, int mx, int my, int mz, int cb,
    const SampleRec* __restrict__ rec, const int4* __restrict__ items, int ntx, int nty,
    int wmode, float2* __restrict__ out, int ldc, int c0, int caller_order) {
  using H = Halo<NDIM>;
  extern __shared__ float lds[];  // [CG][2][PLANE]
  const int4 it = items[blockIdx.x];
  const int tile = it.x, kbeg = it.y, kend = it.z;
  const int cg0 = blockIdx.y * CG, cga = min(CG, cb - cg0);
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int x0 = ix * H::TX, y0 = iy * H::TY, z0 = iz * H::TZ;
  const int tid = threadIdx.x;
  // one thread per voxel of the halo'd tile copies the group's coils, so the
  // index arithmetic is paid once per voxel
  for (int e = tid; e < H::EXT; e += NT) {
    const int lx = e % H::EX, ly = (e / H::EX) % H::EY, lz = e / (H::EX * H::EY);
    // wrap into the grid by subtraction (a runtime modulo costs dozens of
    // instructions): the coordinate is below m + EX - 1 and the grid is at
    // least 4 long per axis, so (EX + 3) / 4 subtractions suffice
    int gx = x0 + lx, gy = y0 + ly, gz = NDIM == 3 ? z0 + lz : 0;
#pragma unroll
    for (int w = 0; w < (H::EX + 3) / 4; ++w) {
      gx -= gx >= mx ? mx : 0;
      gy -= gy >= my ? my : 0;
      if (NDIM == 3) gz -= gz >= mz ? mz : 0;
    }
    const float2* src = G + (((long long)gz * my + gy) * mx + gx) * cb + cg0;
    const int a = lz * H::PZ + ly * H::PY + lx;
#pragma unroll
    for (int q = 0; q < CG; ++q) {
      float2 v = make_float2(0.f, 0.f);
      if (q < cga) v = src[q];
      lds[(size_t)q * 2 * H::PLANE + a] = v.x;
      lds[(size_t)q * 2 * H::PLANE + H::PLANE + a] = v.y;
    }
  }
  __syncthreads();
  for (int k = kbeg + tid; k < kend; k += NT) {
    const SampleRec r = rec[k];
    const int b0 = (NDIM == 3 ? (r.bz - z0) * H::PZ : 0) + (r.by - y0) * H::PY + (r.bx - x0);
    float2 acc[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) acc[q] = make_float2(0.f, 0.f);
    const int nzt = NDIM == 3 ? 4 : 1;
    // one row of four x taps per step: unrolling further lets the compiler
    // hoist the LDS reads of many rows and run out of registers.  The row
    // weights are picked by selects: indexing the record's arrays with a
    // loop counter would put the record in scratch memory.
#pragma unroll 1
    for (int dz = 0; dz < nzt; ++dz) {
      const float wz = NDIM == 3 ? sel4(r.wz, dz) : 1.f;
#pragma unroll 1
      for (int dy = 0; dy < 4; ++dy) {
        const float wyz = wz * sel4(r.wy, dy);
        const int row = b0 + dz * H::PZ + dy * H::PY;
#pragma unroll
        for (int dx = 0; dx < 4; ++dx) {
          const float w = wyz * r.wx[dx];
#pragma unroll
          for (int q = 0; q < CG; ++q) {
            const float* pl = lds + (size_t)q * 2 * H::PLANE + row + dx;
            acc[q].x += w * pl[0];
            acc[q].y += w * pl[H::PLANE];
          }
        }
      }
    }
    const float s = wmode == W_FULL ? r.w : (wmode == W_SQRT ? r.sw : 1.f);
    const long long o = caller_order ? (long long)r.orig : k;
    float2* dst = out + o * ldc + c0 + cg0;
#pragma unroll
    for (int q = 0; q < CG; ++q)
      if (q < cga) dst[q] = make_float2(acc[q].x * s, acc[q].y * s);
  }
}

template <int NDIM, int CG>
size_t interp_tile_lds_bytes() {
  return sizeof(float) * (size_t)CG * 2 * Halo<NDIM>::PLANE;
}

// 512 threads per group in 3D, where the LDS tile allows only one or two
// groups per compute unit
template <int NDIM, int CG>
int interp_tile_launch(cs_ctx* c, const float2* grid, int cb, int wmode, float2* out,
                       int ldc, int c0, int caller_order) {
  const size_t lds = interp_tile_lds_bytes<NDIM, CG>();
  if (lds > 160 * 1024) return fail(c, CS_EINVAL, "interpolation tile does not fit in LDS");
  const int ng = (cb + CG - 1) / CG;
  if (c->n_items == 0) return CS_OK;
  constexpr int NT = NDIM == 3 ? 512 : 256;
  auto kern = k_interp_tile<NDIM, CG, NT>;
  if (lds > 64 * 1024)
    CS_HIP(c, hipFuncSetAttribute((const void*)kern,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  CS_KLAUNCH(c, K_INTERP, kern, dim3((unsigned)c->n_items, (unsigned)ng), dim3(NT), lds,
             c->stream, grid, c->mx, c->my, c->mz, cb, c->rec, c->items, c->ntile[2],
             c->ntile[1], wmode, out, ldc, c0, caller_order);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

// coil groups of at most cmax coils (3D: 8 planar coils of the 11^3 tile
// take 85 KB of LDS, 12 take 128 KB) or 16 (2D); the group size is the chunk
// split evenly
template <int NDIM>
int interp_tile_dispatch(cs_ctx* c, const float2* grid, int cb, int wmode, float2* out,
                         int ldc, int c0, int caller_order, int cmax) {
  if (NDIM == 2) cmax = 16;
  const int ng = (cb + cmax - 1) / cmax;
  const int cg = (cb + ng - 1) / ng;
#define CS_ITILE(CG) \
  return interp_tile_launch<NDIM, CG>(c, grid, cb, wmode, out, ldc, c0, caller_order)
  if (cg <= 2) CS_ITILE(2);
  if (cg <= 4) CS_ITILE(4);
  if (cg <= 6) CS_ITILE(6);
  if (cg <= 8) CS_ITILE(8);
  if (cg <= 12) CS_ITILE(12);
  if constexpr (NDIM == 2) CS_ITILE(16);
#undef CS_ITILE
  return fail(c, CS_EINVAL, "interpolation coil group");
}

constexpr int kSpreadBatch = 64;  // samples staged in LDS per step
// staged record: packed first tap, wx[4], then wy[dy] * wz[dz] at 4 dz + dy
// (the products are formed once per sample in the staging, not by every
// coil wave for every tap)
constexpr int kSpreadRecPitch = 21;

// One work-group = one work item (a contiguous range of the samples of one
// tile, in sorted order) and one group of CG = NW * LPC * CW coils.  Lane l
// of a wave owns tap l % NTAPS of the current sample for CW coils of the
// group.  Consecutive samples with the same first tap touch the same voxels:
// a lane sums such a run in registers and adds the sum into the LDS tile
// once.  The lanes of one LDS instruction address distinct voxels, waves own
// distinct coils, and a wave issues its LDS operations in order, so the
// summation order of every voxel is fixed.  The halo'd tile is written to
// the item's slot; k_spread_merge sums the slots that cover each voxel.
template <int NDIM, int NW, int CW>
__global__ __launch_bounds__(64 * NW) void k_spread(
    const float2* __restrict__ V, int cb, const SampleRec* __restrict__ rec,
    const int4* __restrict__ items, int ntx, int nty, float2* __restrict__ P) {
  using H = Halo<NDIM>;
  constexpr int NT = 64 * NW;
  constexpr int CG = NW * H::LPC * CW;
  constexpr int SB = kSpreadBatch, SRP = kSpreadRecPitch;
  constexpr int VPT = CG * SB / NT;  // staged values per thread
  extern __shared__ float lds[];
  float* acc = lds;                                         // [CG][2][PLANE]
  float* srec = acc + (size_t)CG * 2 * H::PLANE;            // [SB][SRP]
  // staged values: separate re / im planes [SB][2 CG] with the coils two
  // dwords apart, so that every broadcast read below is a single dword
  // (wider same-address LDS reads are much slower on this hardware)
  float* sre = srec + SB * SRP;
  float* sim = sre + SB * 2 * CG;
  __shared__ int s_rs[SB];  // run starts of the staged batch
  __shared__ int s_nr;

  const int4 it = items[blockIdx.x];
  const int tile = it.x, kbeg = it.y, kend = it.z, slot = it.w;
  const int g = blockIdx.y, ng = gridDim.y;
  const int cg0 = g * CG, cga = min(CG, cb - cg0);
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int x0 = ix * H::TX, y0 = iy * H::TY, z0 = iz * H::TZ;
  // the wave index through readfirstlane: the compiler then knows it (and
  // all that depends only on it) to be uniform across the wave
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
            lane = tid & 63;
  for (int i = tid; i < CG * 2 * H::PLANE; i += NT) acc[i] = 0.f;

  const int tap = lane % H::NTAPS, cslot = lane / H::NTAPS;
  const int dx = tap & 3, dy = (tap >> 2) & 3, dz = tap >> 4;
  const int q0 = (wave * H::LPC + cslot) * CW;  // first group coil of this lane
  // waves whose coils all lie beyond the chunk only help with the staging
  const bool active = (wave * H::LPC) * CW < cga;
  float2 racc[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) racc[q] = make_float2(0.f, 0.f);
  int rkey = -1, raddr = 0;

  // staging, double-buffered through registers: thread t < SB fetches the
  // record of sample t of the batch; value e = t + j NT is (sample e / CG,
  // group coil e % CG)
  // (the loaded values are only consumed after the next barrier, so the
  // loads stay in flight while the current batch is processed)
  int pb[3] = {0, 0, 0};
  float pw[12];
  float2 pv[VPT];
  auto prefetch = [&](int k0, int n) {
    if (tid < n) {
      const SampleRec& r = rec[k0 + tid];
      pb[0] = r.bx;
      pb[1] = r.by;
      pb[2] = r.bz;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pw[q] = r.wx[q];
        pw[4 + q] = r.wy[q];
        pw[8 + q] = r.wz[q];
      }
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int e = tid + j * NT, s = e / CG, q = e - s * CG;
      pv[j] = (s < n && q < cga) ? V[(long long)(k0 + s) * cb + cg0 + q]
                                 : make_float2(0.f, 0.f);
    }
  };
  if (kbeg < kend) prefetch(kbeg, min(SB, kend - kbeg));

  for (int k0 = kbeg; k0 < kend; k0 += SB) {
    const int n = min(SB, kend - k0);
    __syncthreads();  // previous batch consumed (and accumulator zeroed)
    const int pkey = (pb[0] - x0) | ((pb[1] - y0) << 8) | ((pb[2] - z0) << 16);
    if (tid < n) {
      float* d = srec + tid * SRP;
      d[0] = __int_as_float(pkey);
#pragma unroll
      for (int q = 0; q < 4; ++q) d[1 + q] = pw[q];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        d[5 + q] = NDIM == 3 ? pw[4 + (q & 3)] * pw[8 + (q >> 2)] : pw[4 + (q & 3)];
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      sre[2 * (tid + j * NT)] = pv[j].x;
      sim[2 * (tid + j * NT)] = pv[j].y;
    }
    // run starts: sample s opens a run when its first tap differs from the
    // previous sample's (or from the run carried over from the last batch)
    if (tid < 64) {
      const int prev = __shfl_up(pkey, 1);
      const bool start = tid < n && pkey != (tid > 0 ? prev : rkey);
      const unsigned long long mask = __ballot(start);
      if (start) s_rs[__popcll(mask & ((1ull << tid) - 1ull))] = tid;
      if (tid == 0) s_nr = __popcll(mask);
    }
    __syncthreads();
    if (k0 + SB < kend) prefetch(k0 + SB, min(SB, kend - k0 - SB));
    // the run bounds are the same for every lane: reading them through
    // readfirstlane keeps the loop control in scalar registers
    const int nr = active ? __builtin_amdgcn_readfirstlane(s_nr) : -1;
    int s = 0;
    for (int r = -1; r < nr; ++r) {
      const int s1 = (r + 1 < nr) ? __builtin_amdgcn_readfirstlane(s_rs[r + 1]) : n;
      if (r >= 0) {
        // close the current run, open the one starting at s
        if (rkey >= 0) {
#pragma unroll
          for (int q = 0; q < CW; ++q) {
            // plain read-add-write: this lane is the only one touching
            // this voxel of this coil until the next flush
            float* pl = acc + (size_t)(q0 + q) * 2 * H::PLANE + raddr;
            pl[0] += racc[q].x;
            pl[H::PLANE] += racc[q].y;
            racc[q] = make_float2(0.f, 0.f);
          }
        }
        rkey = __builtin_amdgcn_readfirstlane(__float_as_int(srec[s * SRP]));
        const int lx = (rkey & 0xff) + dx, ly = ((rkey >> 8) & 0xff) + dy,
                  lz = NDIM == 3 ? (rkey >> 16) + dz : 0;
        raddr = lz * H::PZ + ly * H::PY + lx;
      }
      // samples of the run: register accumulation, no branches
#pragma unroll 4
      for (; s < s1; ++s) {
        const float* d = srec + s * SRP;
        const float w = d[1 + dx] * d[5 + dy + 4 * dz];
        const int vb = 2 * (s * CG + q0);
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          racc[q].x += w * sre[vb + 2 * q];
          racc[q].y += w * sim[vb + 2 * q];
        }
      }
    }
  }
  if (rkey >= 0) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      float* pl = acc + (size_t)(q0 + q) * 2 * H::PLANE + raddr;
      pl[0] += racc[q].x;
      pl[H::PLANE] += racc[q].y;
    }
  }
  __syncthreads();
  // write-out: slot layout [slot][group][EXT][CG]; one thread per voxel
  // writes the group's CG coils of that voxel (contiguous)
  float2* dst = P + ((size_t)slot * ng + g) * H::EXT * CG;
  for (int e = tid; e < H::EXT; e += NT) {
    const int lx = e % H::EX, ly = (e / H::EX) % H::EY, lz = e / (H::EX * H::EY);
    const int a = lz * H::PZ + ly * H::PY + lx;
    float2* d = dst + (size_t)e * CG;
#pragma unroll
    for (int q = 0; q < CG; ++q)
      d[q] = make_float2(acc[(size_t)q * 2 * H::PLANE + a],
                         acc[(size_t)q * 2 * H::PLANE + H::PLANE + a]);
  }
}

// Halo'd tiles that reach grid coordinate g along one axis (tile size T,
// grid length m, nt tiles, g in tile ig): pairs (tile, local coordinate in
// the halo'd tile), in a fixed order.  Returns the count (at most 6).
__device__ __forceinline__ int halo_cover(int g, int ig, int nt, int T, int m, int* ct,
                                          int* cd) {
  int n = 0;
  const int kmax = min(2, nt - 1);
  for (int k = 0; k <= kmax; ++k) {
    int t = ig - k;
    if (t < 0) t += nt;
    const int x0 = t * T, ex = min(T, m - x0);
    int d = g - x0;
    if (d < 0) d += m;
    for (; d < ex + 3 && n < 6; d += m) {
      ct[n] = t;
      cd[n] = d;
      ++n;
    }
  }
  return n;
}

// G = sum of the partial tiles that cover each voxel, in a fixed order
// (covering tile z, y, x, then slot).  One thread per voxel sums all coils;
// every voxel of the grid is written.
template <int NDIM, int CG>
__global__ __launch_bounds__(256) void k_spread_merge(
    const float2* __restrict__ P, const int* __restrict__ item_off, int cb, int ng, int ntx,
    int nty, int ntz, int mx, int my, int mz, float2* __restrict__ G) {
  using H = Halo<NDIM>;
  constexpr int TV = H::TX * H::TY * H::TZ;
  constexpr int BPT = (TV + 255) / 256;  // blocks per tile
  constexpr int NGMAX = (kCoilChunk + CG - 1) / CG;
  const int tile = blockIdx.x / BPT;
  const int v = (blockIdx.x - tile * BPT) * 256 + threadIdx.x;
  if (v >= TV) return;
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int gx = ix * H::TX + v % H::TX, gy = iy * H::TY + (v / H::TX) % H::TY,
            gz = iz * H::TZ + v / (H::TX * H::TY);
  if (gx >= mx || gy >= my || gz >= mz) return;
  int tx[6], dxs[6], ty[6], dys[6], tz[6], dzs[6];
  const int nx_ = halo_cover(gx, ix, ntx, H::TX, mx, tx, dxs);
  const int ny_ = halo_cover(gy, iy, nty, H::TY, my, ty, dys);
  int nz_ = 1;
  tz[0] = 0;
  dzs[0] = 0;
  if (NDIM == 3) nz_ = halo_cover(gz, iz, ntz, H::TZ, mz, tz, dzs);
  float2 acc[NGMAX * CG];
#pragma unroll
  for (int c = 0; c < NGMAX * CG; ++c) acc[c] = make_float2(0.f, 0.f);
  const size_t gstride = (size_t)H::EXT * CG;
  for (int a = 0; a < nz_; ++a)
    for (int b = 0; b < ny_; ++b)
      for (int d = 0; d < nx_; ++d) {
        const int t = (tz[a] * nty + ty[b]) * ntx + tx[d];
        const int e = (dzs[a] * H::EY + dys[b]) * H::EX + dxs[d];
        const int s1 = item_off[t + 1];
        for (int sl = item_off[t]; sl < s1; ++sl) {
          const float2* p = P + (size_t)sl * ng * gstride + (size_t)e * CG;
#pragma unroll
          for (int g = 0; g < NGMAX; ++g) {
            if (g < ng) {
#pragma unroll
              for (int q = 0; q < CG; ++q) {
                const float2 pv = p[g * gstride + q];
                acc[g * CG + q].x += pv.x;
                acc[g * CG + q].y += pv.y;
              }
            }
          }
        }
      }
  float2* out = G + (((long long)gz * my + gy) * mx + gx) * cb;
#pragma unroll
  for (int c = 0; c < NGMAX * CG; ++c)
    if (c < cb) out[c] = acc[c];
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
  if (c->interp_cfg >= 1) {
    const int cmax = c->interp_cfg == 1 ? 8 : (c->interp_cfg == 2 ? 12 : 4);
    return c->ndim == 3
               ? interp_tile_dispatch<3>(c, grid, cb, wmode, out, ldc, c0, caller_order, cmax)
               : interp_tile_dispatch<2>(c, grid, cb, wmode, out, ldc, c0, caller_order, cmax);
  }
  return c->ndim == 3 ? interp_dispatch<3>(c, grid, cb, wmode, out, ldc, c0, caller_order)
                      : interp_dispatch<2>(c, grid, cb, wmode, out, ldc, c0, caller_order);
}

namespace {
template <int NDIM, int NW, int CW>
constexpr int spread_cg() {
  return NW * Halo<NDIM>::LPC * CW;
}

template <int NDIM, int NW, int CW>
size_t spread_lds_bytes() {
  using H = Halo<NDIM>;
  constexpr int CG = spread_cg<NDIM, NW, CW>();
  constexpr int SR = kSpreadBatch * kSpreadRecPitch;
  return sizeof(float) * ((size_t)CG * 2 * H::PLANE + SR + (size_t)4 * kSpreadBatch * CG);
}

template <int NDIM, int NW, int CW>
int spread_launch(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  using H = Halo<NDIM>;
  constexpr int CG = spread_cg<NDIM, NW, CW>();
  const int ng = (cb + CG - 1) / CG;
  if ((size_t)c->n_items * ng * H::EXT * CG > c->partial_elems)
    return fail(c, CS_EINVAL, "spread partial buffer too small");
  const size_t lds = spread_lds_bytes<NDIM, NW, CW>();
  if (lds > 160 * 1024) return fail(c, CS_EINVAL, "spread tile does not fit in LDS");
  if (c->n_items > 0) {
    auto kern = k_spread<NDIM, NW, CW>;
    if (lds > 64 * 1024)
      CS_HIP(c, hipFuncSetAttribute((const void*)kern,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    CS_KLAUNCH(c, K_SPREAD, kern, dim3((unsigned)c->n_items, (unsigned)ng), dim3(64 * NW), lds,
               c->stream, vals, cb, c->rec, c->items, c->ntile[2], c->ntile[1], c->partial);
    CS_HIP(c, hipGetLastError());
  }
  constexpr long long TV = (long long)H::TX * H::TY * H::TZ;
  const long long blocks = c->ntiles * ((TV + 255) / 256);
  if (blocks > 0x7fffffffLL) return fail(c, CS_EINVAL, "spread merge grid too large");
  CS_KLAUNCH(c, K_MERGE, (k_spread_merge<NDIM, CG>), dim3((unsigned)blocks), dim3(256), 0,
             c->stream, c->partial, c->item_off, cb, ng, c->ntile[2], c->ntile[1],
             c->ntile[0], c->mx, c->my, c->mz, grid);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

// work-group shapes (waves NW, coils per lane CW); the coils of a group are
// NW * CW (3D) or 4 NW CW (2D, four coil slots of 16 taps per wave)
template <int NDIM>
int spread_dispatch(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  switch (c->spread_cfg) {
    case 1: return spread_launch<NDIM, 2, 2>(c, vals, cb, grid);
    case 2: return spread_launch<NDIM, 2, 1>(c, vals, cb, grid);
    case 3: return spread_launch<NDIM, 1, 4>(c, vals, cb, grid);
    case 4: return spread_launch<NDIM, 4, 2>(c, vals, cb, grid);
    case 5: return spread_launch<NDIM, 1, 3>(c, vals, cb, grid);
    case 6:
      // all coils of the chunk in one work-group where the LDS allows (one
      // wave per coil), so every sample is staged once
      if constexpr (NDIM == 3) {
        if (cb <= 4) return spread_launch<NDIM, 4, 1>(c, vals, cb, grid);
        if (cb <= 6) return spread_launch<NDIM, 6, 1>(c, vals, cb, grid);
        if (cb <= 8) return spread_launch<NDIM, 8, 1>(c, vals, cb, grid);
        if (cb <= 12) return spread_launch<NDIM, 12, 1>(c, vals, cb, grid);
        return spread_launch<NDIM, 8, 1>(c, vals, cb, grid);
      } else {
        return spread_launch<NDIM, 4, 1>(c, vals, cb, grid);
      }
    default: return spread_launch<NDIM, 4, 1>(c, vals, cb, grid);
  }
}

// largest coil-group size over the shapes above, for the partial buffer
int spread_max_group_elems(int ndim) {
  const int lpc = ndim == 3 ? 1 : 4;
  const int cgs[6] = {4 * lpc, 4 * lpc, 2 * lpc, 4 * lpc, 8 * lpc, 3 * lpc};
  int best = 0;
  for (int cg : cgs) best = std::max(best, ((kCoilChunk + cg - 1) / cg) * cg);
  return best;
}
}  // namespace

int launch_spread(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "spread coil chunk");
  return c->ndim == 3 ? spread_dispatch<3>(c, vals, cb, grid)
                      : spread_dispatch<2>(c, vals, cb, grid);
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
  if (N > 0x7fffffffLL) return fail(c, CS_EINVAL, "more than 2^31 - 1 samples");
  std::vector<float> coords((size_t)N * nd), dcf;
  if (N > 0)
    CS_HIP(c, hipMemcpy(coords.data(), coords_dev, sizeof(float) * N * nd,
                        hipMemcpyDeviceToHost));
  if (N == 0) dcf_dev = nullptr;  // empty trajectory: the zero operator
  if (dcf_dev) {
    dcf.resize(N);
    CS_HIP(c, hipMemcpy(dcf.data(), dcf_dev, sizeof(float) * N, hipMemcpyDeviceToHost));
    for (long long i = 0; i < N; ++i)
      if (!(dcf[i] >= 0.f)) return fail(c, CS_EINVAL, "density compensation must be >= 0");
  }
  const int n[3] = {c->nz, c->ny, c->nx};
  const int m[3] = {c->mz, c->my, c->mx};
  const double W = 4.0, beta = c->beta;

  // spread tiles: 8x8x8 (3D) or 16x16 (2D) voxels; the work-group shape is
  // a tuning knob (CS_SPREAD_CFG in the environment, see spread_dispatch)
  c->tile[0] = nd == 3 ? 8 : 1;
  c->tile[1] = nd == 3 ? 8 : 16;
  c->tile[2] = nd == 3 ? 8 : 16;
  for (int a = 3 - nd; a < 3; ++a)
    if (m[a] < 4) return fail(c, CS_EINVAL, "NUFFT grid shorter than the kernel");
  const char* cfg = std::getenv("CS_SPREAD_CFG");
  c->spread_cfg = cfg ? std::atoi(cfg) : 0;
  const char* icfg = std::getenv("CS_INTERP_CFG");
  c->interp_cfg = icfg ? std::atoi(icfg) : 1;
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

  // samples per tile (each sample belongs to the tile of its first tap)
  std::vector<long long> toff(c->ntiles + 1, 0);
  for (long long j = 0; j < N; ++j) toff[(key[order[j]] >> 40) + 1]++;
  for (long long t = 0; t < c->ntiles; ++t) toff[t + 1] += toff[t];

  CS_HIP(c, hipMalloc(&c->rec, sizeof(SampleRec) * std::max(1LL, N)));
  if (N > 0)
    CS_HIP(c, hipMemcpy(c->rec, srec.data(), sizeof(SampleRec) * N, hipMemcpyHostToDevice));
  if (dcf_dev) {
    CS_HIP(c, hipMalloc(&c->dcf_orig, sizeof(float) * N));
    CS_HIP(c, hipMemcpy(c->dcf_orig, dcf.data(), sizeof(float) * N, hipMemcpyHostToDevice));
  }

  // spread work items: each tile's samples in chunks of at most `chunk`; the
  // slot of an item is its index in tile order, so the slots of tile t are
  // item_off[t] .. item_off[t + 1]
  const long long chunk = 2048;
  std::vector<int4> items;
  std::vector<int> ioff(c->ntiles + 1, 0);
  for (long long t = 0; t < c->ntiles; ++t) {
    for (long long k = toff[t]; k < toff[t + 1]; k += chunk) {
      const int slot = (int)items.size();
      items.push_back(make_int4((int)t, (int)k, (int)std::min(toff[t + 1], k + chunk), slot));
    }
    ioff[t + 1] = (int)items.size();
  }
  // heavy items first so that the long ones start early
  std::stable_sort(items.begin(), items.end(),
                   [](const int4& a, const int4& b) { return (a.z - a.y) > (b.z - b.y); });
  c->n_items = (long long)items.size();
  CS_HIP(c, hipMalloc(&c->items, sizeof(int4) * std::max<size_t>(1, items.size())));
  if (!items.empty())
    CS_HIP(c, hipMemcpy(c->items, items.data(), sizeof(int4) * items.size(),
                        hipMemcpyHostToDevice));
  CS_HIP(c, hipMalloc(&c->item_off, sizeof(int) * ioff.size()));
  CS_HIP(c, hipMemcpy(c->item_off, ioff.data(), sizeof(int) * ioff.size(),
                      hipMemcpyHostToDevice));
  const size_t ext = nd == 3 ? (size_t)Halo<3>::EXT : (size_t)Halo<2>::EXT;
  c->partial_elems = std::max<size_t>(1, (size_t)c->n_items * ext * spread_max_group_elems(nd));
  CS_HIP(c, hipMalloc(&c->partial, sizeof(float2) * c->partial_elems));
  return CS_OK;
}

}  // namespace cs
