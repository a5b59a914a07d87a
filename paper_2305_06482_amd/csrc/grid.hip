// Kaiser-Bessel gridding for the non-uniform FFT of Sec. 2.1 (F~ = F~_n,
// implemented as a NUFFT after Beatty et al. 2005) with density compensation
// A = W^1/2 F C (Sec. 2.1.1).
//
// Set-up (once per operator, host): each sample's grid coordinate
// u_a = k_a m_a / n_a gives its first tap floor(u_a) - 1 (wrapped into the
// grid).  Samples are sorted by the 8x8x8 (3D) or 16x16 (2D) grid tile that
// holds their first tap, then by that tap, and each tile's samples are cut
// into work items of at most 2048 samples.  A sample's 64-byte record holds
// its first tap relative to the tile's origin (packed), w, sqrt(w), its index
// in the caller's order and the four kernel weights phi(u_a - g) per axis,
// evaluated in FP64 and stored as FP32.
//
// interp: one work-group per work item and coil group copies the item's
//         halo'd grid tile (the tile grown by the kernel's 3-voxel reach,
//         wrapped modulo the grid) into LDS and sums each sample's 4^d taps
//         from there (one thread per sample).
// spread: one work-group per work item and coil group accumulates, in LDS,
//         its samples into the halo'd tile (each sample is handled once),
//         one sample at a time with one lane per tap.  Within a LDS
//         instruction all lanes address distinct voxels and a wave executes
//         its LDS instructions in order, so every voxel's summation order is
//         fixed.  The halo'd tile is written to the item's slot, and a merge
//         kernel sums, for every grid voxel, the slots that cover it in a
//         fixed order: deterministic, and no global atomics.
// The normal operator W^1/2 W^1/2 between the transforms (Eq. 5) runs
// interp (x w) and spread over groups of work items whose sample values fit
// a fixed buffer, so that the values one group's interpolation writes are
// read back by its spreading from the on-chip caches.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <type_traits>
#include <utility>

#include "cs_internal.h"

namespace cs {

// I0 by its power series sum (x^2/4)^k / (k!)^2 (converges for all x; the
// argument here is at most beta ~ 7).  Host and device evaluate it (and the
// kernel below) with the same operations and no contraction into FMAs, so the
// set-up's weights do not depend on where they are computed.
__host__ __device__ double kb_i0_hd(double x) {
#pragma clang fp contract(off)
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

double kb_i0(double x) { return kb_i0_hd(x); }

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

__host__ __device__ double kb_kernel(double t, double W, double beta) {
#pragma clang fp contract(off)
  const double z = 1.0 - (2.0 * t / W) * (2.0 * t / W);
  return z >= 0 ? kb_i0_hd(beta * sqrt(z)) : 0.0;
}

__device__ __forceinline__ float sel4(const float* w, int i) {
  return i == 0 ? w[0] : (i == 1 ? w[1] : (i == 2 ? w[2] : w[3]));
}

// Halo'd spread tile: every sample belongs to the one tile that holds its
// first tap, and its 4^d footprint stays inside the tile grown by 3 voxels
// along each axis.  The LDS tiles are planar per (coil, re/im) with voxel
// offset lz * PZ + ly * PY + lx: dense in 3D (the 64 taps of a sample meet
// at most two per bank, and only when a run is flushed) and with row pitch
// 20 in 2D (16 taps in distinct banks).
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

// Work item (relative to item0) and coil group of this work-group.  With a
// two-dimensional grid (items, groups) they are blockIdx.x and blockIdx.y.
// With xcd the grid is one-dimensional and the coil groups of item i sit at
// blocks 8 (ng (i / 8) + g) + i % 8: work-groups are dealt to the 8 XCDs in
// turn, so all groups of an item run on one XCD, close together in time,
// and every group after the first finds the item's sample records (and, for
// the interpolation, its grid tile) in that XCD's L2.  False for the padding
// blocks past the last item.
__device__ __forceinline__ bool item_and_group(int nitems, int ng, int xcd, int& item,
                                               int& g) {
  if (!xcd) {
    item = blockIdx.x;
    g = blockIdx.y;
    return true;
  }
  const int b = blockIdx.x, t = b >> 3;
  g = t % ng;
  item = (t / ng) * 8 + (b & 7);
  return item < nitems;
}

inline dim3 item_group_grid(long long nitems, int ng, int xcd) {
  return xcd ? dim3((unsigned)(((nitems + 7) / 8) * 8 * ng)) : dim3((unsigned)nitems, (unsigned)ng);
}

// Interpolation: one work-group per work item and coil group.  With TILE the
// group first copies the item's halo'd tile of the grid into LDS, planar per
// (coil, re/im) as in the spreading accumulator; without it the taps are
// read from the grid in global memory.  One thread per sample then sums its
// 4^d taps in the order z, y, x with weight (wz wy) wx, so both variants give
// the same values.  The sum is scaled by w (W_FULL), sqrt(w) (W_SQRT) or 1,
// and written to row `voff + k - kbeg` of `out` (values of the item group)
// or, with caller_order, to row orig[k] (the caller's sample order).  With
// vec (even cb, ldc and c0, 16-byte aligned G and out), a full group moves
// its coils two at a time, 16 bytes per access.
template <int NDIM, int CG, int NT, bool TILE, bool IL = false>
__global__ __launch_bounds__(NT) void k_interp_items(
    const float2* __restrict__ G, int mx, int my, int mz, int cb,
    const SampleRec* __restrict__ rec, const GridItem* __restrict__ items, int item0,
    int ntx, int nty, int wmode, float2* __restrict__ out, int ldc, int c0,
    int caller_order, int nitems, int xcd, int vec) {
  using H = Halo<NDIM>;
  extern __shared__ float lds[];  // [CG][2][PLANE]
  int item, grp;
  if (!item_and_group(nitems, (cb + CG - 1) / CG, xcd, item, grp)) return;
  const GridItem it = items[item0 + item];
  const int tile = it.tile, kbeg = it.kbeg, kend = it.kend;
  const int cg0 = grp * CG, cga = min(CG, cb - cg0);
  const bool v2 = CG % 2 == 0 && vec && cga == CG;
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int x0 = ix * H::TX, y0 = iy * H::TY, z0 = iz * H::TZ;
  const int tid = threadIdx.x;
  // this thread's first sample record, requested before the tile so that
  // the two loads overlap
  SampleRec r0;
  if (kbeg + tid < kend) r0 = rec[kbeg + tid];
  if constexpr (TILE) {
    // one thread per voxel of the halo'd tile copies the group's coils, so
    // the index arithmetic is paid once per voxel; a thread's voxels are
    // loaded in one unrolled sweep, then stored to LDS
    constexpr int NE = (H::EXT + NT - 1) / NT;
    float2 tv[NE][CG];
    int ta[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * NT;
      ta[i] = -1;
      if (e < H::EXT) {
        const int lx = e % H::EX, ly = (e / H::EX) % H::EY, lz = e / (H::EX * H::EY);
        // wrap into the grid by subtraction (a runtime modulo costs dozens
        // of instructions): the coordinate is below m + EX - 1 and the grid
        // is at least 4 long per axis, so (EX + 3) / 4 subtractions suffice
        int gx = x0 + lx, gy = y0 + ly, gz = NDIM == 3 ? z0 + lz : 0;
#pragma unroll
        for (int w = 0; w < (H::EX + 3) / 4; ++w) {
          gx -= gx >= mx ? mx : 0;
          gy -= gy >= my ? my : 0;
          if (NDIM == 3) gz -= gz >= mz ? mz : 0;
        }
        const float2* src = G + (((long long)gz * my + gy) * mx + gx) * cb + cg0;
        ta[i] = lz * H::PZ + ly * H::PY + lx;
        if (v2) {
#pragma unroll
          for (int q = 0; q < CG / 2; ++q) {
            const float4 t = reinterpret_cast<const float4*>(src)[q];
            tv[i][2 * q] = make_float2(t.x, t.y);
            tv[i][2 * q + 1] = make_float2(t.z, t.w);
          }
        } else {
#pragma unroll
          for (int q = 0; q < CG; ++q) tv[i][q] = q < cga ? src[q] : make_float2(0.f, 0.f);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      if (ta[i] < 0) continue;
      const int a = ta[i];
#pragma unroll
      for (int q = 0; q < CG; ++q) {
        if constexpr (IL) {
          // interleaved (re, im) per voxel: one 8-byte LDS read per tap
          reinterpret_cast<float2*>(lds)[(size_t)q * H::PLANE + a] = tv[i][q];
        } else {
          lds[(size_t)q * 2 * H::PLANE + a] = tv[i][q].x;
          lds[(size_t)q * 2 * H::PLANE + H::PLANE + a] = tv[i][q].y;
        }
      }
    }
    __syncthreads();
  }
  SampleRec r = r0;
  for (int k = kbeg + tid; k < kend; k += NT) {
    if (k != kbeg + tid) r = rec[k];
    const int lx = r.key & 0xff, ly = (r.key >> 8) & 0xff, lz = r.key >> 16;
    float2 acc[CG];
#pragma unroll
    for (int q = 0; q < CG; ++q) acc[q] = make_float2(0.f, 0.f);
    const int nzt = NDIM == 3 ? 4 : 1;
    // one row of four x taps per step (two rows for groups of at most 4
    // coils): unrolling further lets the compiler hoist the reads of many
    // rows and run out of registers.  The row weights are picked by selects:
    // indexing the weight arrays with a loop counter would put them in
    // scratch memory.
    constexpr int UY = CG <= 4 ? 2 : 1;
#pragma unroll 1
    for (int dz = 0; dz < nzt; ++dz) {
      const float wzv = NDIM == 3 ? sel4(r.wz, dz) : 1.f;
#pragma unroll UY
      for (int dy = 0; dy < 4; ++dy) {
        const float wyz = wzv * sel4(r.wy, dy);
        if constexpr (TILE) {
          const int row = (lz + dz) * H::PZ + (ly + dy) * H::PY + lx;
#pragma unroll
          for (int dx = 0; dx < 4; ++dx) {
            const float w = wyz * r.wx[dx];
#pragma unroll
            for (int q = 0; q < CG; ++q) {
              if constexpr (IL) {
                const float2 g = reinterpret_cast<const float2*>(lds)[(size_t)q * H::PLANE + row + dx];
                acc[q].x += w * g.x;
                acc[q].y += w * g.y;
              } else {
                const float* pl = lds + (size_t)q * 2 * H::PLANE + row + dx;
                acc[q].x += w * pl[0];
                acc[q].y += w * pl[H::PLANE];
              }
            }
          }
        } else {
          // the first tap x0 + lx lies in [0, m) and m >= 4: one subtraction
          // wraps a tap
          int z = z0 + lz + dz, y = y0 + ly + dy;
          if (NDIM == 3) z -= z >= mz ? mz : 0;
          y -= y >= my ? my : 0;
          const long long rowg = ((long long)(NDIM == 3 ? z : 0) * my + y) * mx;
#pragma unroll
          for (int dx = 0; dx < 4; ++dx) {
            const float w = wyz * r.wx[dx];
            int x = x0 + lx + dx;
            x -= x >= mx ? mx : 0;
            const float2* p = G + (rowg + x) * cb + cg0;
#pragma unroll
            for (int q = 0; q < CG; ++q) {
              if (q < cga) {
                const float2 g = p[q];
                acc[q].x += w * g.x;
                acc[q].y += w * g.y;
              }
            }
          }
        }
      }
    }
    const float s = wmode == W_FULL ? r.w : (wmode == W_SQRT ? r.sw : 1.f);
    const long long o = caller_order ? (long long)r.orig : (long long)(it.voff + k - kbeg);
    float2* dst = out + o * ldc + c0 + cg0;
    if (v2) {
#pragma unroll
      for (int q = 0; q < CG / 2; ++q)
        reinterpret_cast<float4*>(dst)[q] = make_float4(acc[2 * q].x * s, acc[2 * q].y * s,
                                                        acc[2 * q + 1].x * s,
                                                        acc[2 * q + 1].y * s);
    } else {
#pragma unroll
      for (int q = 0; q < CG; ++q)
        if (q < cga) dst[q] = make_float2(acc[q].x * s, acc[q].y * s);
    }
  }
}

template <int NDIM, int CG>
size_t interp_tile_lds_bytes() {
  return sizeof(float) * (size_t)CG * 2 * Halo<NDIM>::PLANE;
}

// 512 threads per group in 3D, where the LDS tile allows only one or two
// groups per compute unit
template <int NDIM, int CG, bool TILE, bool IL = false>
int interp_launch(cs_ctx* c, const float2* grid, int cb, int item0, int nitems, int wmode,
                  float2* out, int ldc, int c0, int caller_order) {
  const size_t lds = TILE ? interp_tile_lds_bytes<NDIM, CG>() : 0;
  if (lds > 160 * 1024) return fail(c, CS_EINVAL, "interpolation tile does not fit in LDS");
  const int ng = (cb + CG - 1) / CG;
  if (nitems <= 0) return CS_OK;
  constexpr int NT = NDIM == 3 ? 512 : 256;
  auto kern = k_interp_items<NDIM, CG, NT, TILE, IL>;
  if (lds > 64 * 1024)
    CS_HIP(c, hipFuncSetAttribute((const void*)kern,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int vec = c->grid_vec && cb % 2 == 0 && ldc % 2 == 0 && c0 % 2 == 0 &&
                  ((uintptr_t)grid & 15) == 0 && ((uintptr_t)out & 15) == 0;
  CS_KLAUNCH(c, K_INTERP, kern, item_group_grid(nitems, ng, c->grid_xcd), dim3(NT), lds,
             c->stream, grid, c->mx, c->my, c->mz, cb, c->rec, c->gitems, item0, c->ntile[2],
             c->ntile[1], wmode, out, ldc, c0, caller_order, nitems, c->grid_xcd, vec);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

// coil groups of at most cmax coils (3D: 8 planar coils of the 11^3 tile
// take 85 KB of LDS, 12 take 128 KB) or 16 (2D); the group size is the chunk
// split evenly.  Variant 0 reads the grid in global memory (groups of 8).
template <int NDIM>
int interp_dispatch(cs_ctx* c, const float2* grid, int cb, int item0, int nitems, int wmode,
                    float2* out, int ldc, int c0, int caller_order) {
  const bool tile = c->interp_cfg >= 1;
  const bool il = c->interp_cfg == 4;  // interleaved (re, im) LDS tile
  int cmax = c->interp_cfg == 2 ? 12 : (c->interp_cfg >= 3 ? 4 : 8);
  if (NDIM == 2) cmax = 16;
  const int ng = (cb + cmax - 1) / cmax;
  const int cg = (cb + ng - 1) / ng;
#define CS_ITILE(CG)                                                                        \
  return il ? interp_launch<NDIM, CG, true, true>(c, grid, cb, item0, nitems, wmode, out,  \
                                                  ldc, c0, caller_order)                   \
       : tile ? interp_launch<NDIM, CG, true>(c, grid, cb, item0, nitems, wmode, out, ldc, \
                                              c0, caller_order)                            \
              : interp_launch<NDIM, CG, false>(c, grid, cb, item0, nitems, wmode, out,     \
                                               ldc, c0, caller_order)
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
// default spreading shape: register-held values and kernel weights, values
// broadcast by DPP, 4 waves of one coil each (shape 12 of spread_dispatch)
constexpr int kSpreadDefault = 12;
// staged record: packed first tap, wx[4], then wy[dy] * wz[dz] at 4 dz + dy
// (the products are formed once per sample in the staging, not by every
// coil wave for every tap)
constexpr int kSpreadRecPitch = 21;
enum { SRC_VALS = 0, SRC_DATA = 1 };

// f(std::integral_constant<int, i>) for i = 0 .. N-1, expanded at compile time
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// acc += src[lane j of this lane's row of 16] * w: a VOP2 FMA whose first
// operand is read through the row broadcast of DPP (row_newbcast, CDNA3 and
// later), so a value is broadcast and used in one instruction
template <int J>
__device__ __forceinline__ void fmac_rowbcast(float& acc, float src, float w) {
  asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(acc)
               : "v"(src), "v"(w), "n"(J));
}

// One batch of the register-weight spreading (k_spread_rl VAR 2 and 3,
// k_spread_items with RW): every lane forms its tap's weight for all
// samples of the batch in registers, then one pass over the batch, expanded
// at compile time (the weight register and, with DPP, the broadcast lane
// are constants of each step), takes the run starts from the bit mask
// sm1:sm0 and keeps the run state (racc, rbase, rkey, raddr) across batches.
// Values: with DPP chunk c of 16 samples in cr[q][c] (sample 16 c + j in
// lane j of every row of 16), else sample j's in lane j of cv[q].  Lanes
// beyond the staged rows form weights from stale records, never used.
// lacc = this lane's tap of its first coil plane at the tile origin; rp =
// the open run's voxel in that plane (coil q at rp + 2 q PLANE).
template <int NDIM, int CW, bool DPP>
__device__ __forceinline__ void rw_batch(float* lacc, const float* srec, int n, unsigned sm0,
                                         unsigned sm1, int vkey, int dx, int dy, int dz,
                                         bool active, const float2 (&cr)[CW][4],
                                         const float2 (&cv)[CW], float2 (&racc)[CW],
                                         float2 (&rbase)[CW], int& rkey, float*& rp) {
  using H = Halo<NDIM>;
  constexpr int SB = kSpreadBatch, SRP = kSpreadRecPitch;
  // rows s >= n hold stale records: their weights are formed, never
  // used.  All reads are issued before the first product; the empty asm
  // statements keep the products ahead of the sample loop (rather than
  // inside its run branches)
  float wr[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const float* d = srec + s * SRP;
    wr[s] = d[1 + dx] * d[5 + dy + 4 * dz];
  }
#pragma unroll
  for (int s = 0; s < SB; ++s) asm volatile("" : "+v"(wr[s]));
  if (!active) return;
  // one step per sample, expanded at compile time (the broadcast lane
  // and the weight register are constants of each step); a full batch
  // (the usual case) runs a copy without the per-sample bound test
  auto step = [&](auto sc, auto fc) {
    constexpr int s = decltype(sc)::value;
    if constexpr (!decltype(fc)::value) {
      if (s >= n) return;
    }
    if (((s < 32 ? sm0 : sm1) >> (s & 31)) & 1u) {
      // the LDS value of the run's voxel was read when the run opened
      // (a run's voxels are this lane's alone until it flushes), so
      // the flush rarely waits
      // no test for an open run: before the item's first run rp is the
      // tile origin of this lane's tap and rbase = racc = 0, and the LDS tile
      // is still all zero there, so that flush writes 0 over 0 (one code path
      // also spares the wait that the merge of two paths would put before
      // the next run's reads)
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        float* pl = rp + (size_t)q * 2 * H::PLANE;
        pl[0] = rbase[q].x + racc[q].x;
        pl[H::PLANE] = rbase[q].y + racc[q].y;
        racc[q] = make_float2(0.f, 0.f);
      }
      rkey = __builtin_amdgcn_readlane(vkey, s);
      // the run's first tap is uniform: a scalar offset, one vector add
      rp = lacc + __builtin_amdgcn_readfirstlane((rkey >> 16) * H::PZ +
                                                 ((rkey >> 8) & 0xff) * H::PY + (rkey & 0xff));
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const float* pl = rp + (size_t)q * 2 * H::PLANE;
        rbase[q] = make_float2(pl[0], pl[H::PLANE]);
      }
    }
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      if constexpr (DPP) {
        fmac_rowbcast<(s & 15)>(racc[q].x, cr[q][s >> 4].x, wr[s]);
        fmac_rowbcast<(s & 15)>(racc[q].y, cr[q][s >> 4].y, wr[s]);
      } else {
        const float vr =
            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv[q].x), s));
        const float vi =
            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv[q].y), s));
        racc[q].x += wr[s] * vr;
        racc[q].y += wr[s] * vi;
      }
    }
  };
  auto run = [&](auto fc) {
    auto one = [&](auto sc) { step(sc, fc); };
    static_for<SB>(one);
  };
  if (n == SB)
    run(std::true_type{});
  else
    run(std::false_type{});
}

// One work-group = one work item (a contiguous range of the samples of one
// tile, in sorted order) and one group of CG = NW * LPC * CW coils.  Lane l
// of a wave owns tap l % NTAPS of the current sample for CW coils of the
// group.  Consecutive samples with the same first tap touch the same voxels:
// a lane sums such a run in registers and adds the sum into the LDS tile
// once.  The lanes of one LDS instruction address distinct voxels, waves own
// distinct coils, and a wave issues its LDS operations in order, so the
// summation order of every voxel is fixed.  The halo'd tile is written to
// the item's slot; k_spread_merge sums the slots that cover each voxel.
// Sample values come from `V`: with SRC_VALS row voff + (k - kbeg) of the
// item group's values (cb coils per row); with SRC_DATA the caller's data
// row orig (coils c0 .. at leading dimension ldc), scaled by sqrt(w)
// (folded into the staged x weights).
// With RW the batch runs through rw_batch (kernel weights in registers,
// values by DPP row broadcasts; every row of 16 lanes is one coil slot in
// 2D, so a row broadcast hands each slot its own coil's value).
template <int NDIM, int NW, int CW, int SRC, bool RW = false>
__global__ __launch_bounds__(64 * NW) void k_spread_items(
    const float2* __restrict__ V, int ldc, int c0, int cb, const SampleRec* __restrict__ rec,
    const GridItem* __restrict__ items, int item0, int ntx, int nty,
    float2* __restrict__ P, int nitems, int xcd) {
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
  __shared__ unsigned s_sm[2];  // the run starts as a bit mask (RW)

  const int ng = (cb + CG - 1) / CG;
  int item, g;
  if (!item_and_group(nitems, ng, xcd, item, g)) return;
  const GridItem it = items[item0 + item];
  const int tile = it.tile, kbeg = it.kbeg, kend = it.kend, slot = it.slot;
  const int cg0 = g * CG, cga = min(CG, cb - cg0);
  // the wave index through readfirstlane: the compiler then knows it (and
  // all that depends only on it) to be uniform across the wave
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
            lane = tid & 63;
  for (int i = tid; i < CG * 2 * H::PLANE; i += NT) acc[i] = 0.f;

  const int tap = lane % H::NTAPS, cslot = lane / H::NTAPS;
  const int dx = tap & 3, dy = (tap >> 2) & 3, dz = tap >> 4;
  const int loff = dz * H::PZ + dy * H::PY + dx;  // this lane's tap in the tile
  const int q0 = (wave * H::LPC + cslot) * CW;  // first group coil of this lane
  // waves whose coils all lie beyond the chunk only help with the staging
  const bool active = (wave * H::LPC) * CW < cga;
  float2 racc[CW], rbase[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) racc[q] = rbase[q] = make_float2(0.f, 0.f);
  int rkey = -1, raddr = 0;
  float* const lacc = acc + (size_t)q0 * 2 * H::PLANE + loff;  // RW run addressing
  float* rp = lacc;

  // staging, double-buffered through registers: thread t < SB fetches the
  // record of sample t of the batch; value e = t + j NT is (sample e / CG,
  // group coil e % CG).  The loaded values are only consumed after the next
  // barrier, so the loads stay in flight while the current batch is
  // processed.
  int pkey = 0;
  float pw[12], psw = 1.f;
  float2 pv[VPT];
  auto prefetch = [&](int k0, int n) {
    if (tid < n) {
      const SampleRec& r = rec[k0 + tid];
      pkey = r.key;
      psw = r.sw;
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
      float2 v = make_float2(0.f, 0.f);
      if (s < n && q < cga) {
        if constexpr (SRC == SRC_VALS)
          v = V[(long long)(it.voff + k0 - kbeg + s) * cb + cg0 + q];
        else
          v = V[(long long)rec[k0 + s].orig * ldc + c0 + cg0 + q];
      }
      pv[j] = v;
    }
  };
  if (kbeg < kend) prefetch(kbeg, min(SB, kend - kbeg));

  for (int k0 = kbeg; k0 < kend; k0 += SB) {
    const int n = min(SB, kend - k0);
    __syncthreads();  // previous batch consumed (and accumulator zeroed)
    if (tid < n) {
      // x weights (times sqrt(w) for caller data), then wy[dy] wz[dz]
      const float sx = SRC == SRC_DATA ? psw : 1.f;
      float* d = srec + tid * SRP;
      d[0] = __int_as_float(pkey);
#pragma unroll
      for (int q = 0; q < 4; ++q) d[1 + q] = pw[q] * sx;
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
      if (tid == 0) {
        s_nr = __popcll(mask);
        s_sm[0] = (unsigned)mask;
        s_sm[1] = (unsigned)(mask >> 32);
      }
    }
    __syncthreads();
    if constexpr (RW) {
      static_assert(SB == 64, "one run-start bit per sample");
      // chunk c of 16 samples: sample 16 c + (lane & 15) of this lane's coil
      float2 cr[CW][4], cv[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        cv[q] = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int e = 2 * ((16 * c + (lane & 15)) * CG + q0 + q);
          cr[q][c] = make_float2(sre[e], sim[e]);
        }
      }
      const int vkey = __float_as_int(srec[lane * SRP]);
      const unsigned sm0 = __builtin_amdgcn_readfirstlane(s_sm[0]),
                     sm1 = __builtin_amdgcn_readfirstlane(s_sm[1]);
      if (k0 + SB < kend) prefetch(k0 + SB, min(SB, kend - k0 - SB));
      rw_batch<NDIM, CW, true>(lacc, srec, n, sm0, sm1, vkey, dx, dy, dz, active, cr, cv, racc,
                               rbase, rkey, rp);
      continue;
    }
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
        // the run's first tap is uniform: its offset is scalar arithmetic,
        // and one vector add places this lane's tap
        const int lz = NDIM == 3 ? (rkey >> 16) : 0;
        raddr = __builtin_amdgcn_readfirstlane(lz * H::PZ + ((rkey >> 8) & 0xff) * H::PY +
                                               (rkey & 0xff)) + loff;
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
      float* pl = RW ? rp + (size_t)q * 2 * H::PLANE
                     : acc + (size_t)(q0 + q) * 2 * H::PLANE + raddr;
      if constexpr (RW) {
        pl[0] = rbase[q].x + racc[q].x;
        pl[H::PLANE] = rbase[q].y + racc[q].y;
      } else {
        pl[0] += racc[q].x;
        pl[H::PLANE] += racc[q].y;
      }
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

// The 3D spreading of the normal operator with the sample values held in
// vector registers instead of LDS: lane j of a wave keeps sample j's values
// of the wave's CW coils, and each sample's values are broadcast to the
// wave's lanes by v_readlane into scalar registers that enter the FMAs as
// scalar operands.  Only the kernel weights go through LDS.  Summation
// order as in k_spread_items (bit-identical results).
// VAR 0: a loop over the batch's runs, the weights read from LDS per sample;
// VAR 1: the same, and the LDS value of a run's voxel is read when the run
// opens, so that its flush only adds and writes;
// VAR 2: every lane first forms its tap's weight for all samples of the
// batch in registers, then one pass over the batch, unrolled so that the
// weights are static register operands, takes the run starts from a bit
// mask; no LDS access in the sample loop outside the run flushes, which
// work as in VAR 1;
// VAR 3: VAR 2 with the values broadcast by DPP instead of v_readlane: every
// row of 16 lanes holds the values of the same 16 samples, and the FMA
// reads sample j's through row_newbcast:j (one instruction per product).
// (LDS admits at most three waves per SIMD; the register budget is held to
// that occupancy.)
template <int NW, int CW, int VAR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void k_spread_rl(
    const float2* __restrict__ V, int /*ldc*/, int /*c0*/, int cb,
    const SampleRec* __restrict__ rec,
    const GridItem* __restrict__ items, int item0, int ntx, int nty,
    float2* __restrict__ P, int nitems, int xcd) {
  using H = Halo<3>;
  constexpr int NT = 64 * NW;
  constexpr int CG = NW * CW;
  constexpr int SB = kSpreadBatch, SRP = kSpreadRecPitch;
  extern __shared__ float lds[];
  float* acc = lds;                               // [CG][2][PLANE]
  float* srec = acc + (size_t)CG * 2 * H::PLANE;  // [SB][SRP]
  __shared__ int s_rs[SB];
  __shared__ int s_nr;
  __shared__ unsigned s_sm[2];  // run starts of the batch as a bit mask
  constexpr bool PF = VAR >= 1;  // run's voxel read when it opens

  const int ng = (cb + CG - 1) / CG;
  int item, g;
  if (!item_and_group(nitems, ng, xcd, item, g)) return;
  const GridItem it = items[item0 + item];
  const int tile = it.tile, kbeg = it.kbeg, kend = it.kend, slot = it.slot;
  const int cg0 = g * CG, cga = min(CG, cb - cg0);
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
            lane = tid & 63;
  for (int i = tid; i < CG * 2 * H::PLANE; i += NT) acc[i] = 0.f;

  const int dx = lane & 3, dy = (lane >> 2) & 3, dz = lane >> 4;
  const int loff = dz * H::PZ + dy * H::PY + dx;  // this lane's tap in the tile
  const int q0 = wave * CW;  // first group coil of this wave
  const bool active = q0 < cga;
  float2 racc[CW];
  // PF: the LDS value of the run's voxel, read when the run opens (the lane
  // owns the voxel until it flushes), so the flush only adds and writes
  float2 rbase[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) racc[q] = rbase[q] = make_float2(0.f, 0.f);
  int rkey = -1, raddr = 0;
  float* const lacc = acc + (size_t)q0 * 2 * H::PLANE + loff;  // VAR >= 2 run addressing
  float* rp = lacc;

  // thread t < SB fetches the record of sample t of the next batch; lane j of
  // every wave fetches sample j's values of the wave's coils, which pass
  // through this wave's slice of LDS once per batch (so that no load is in
  // flight while the loop below broadcasts them)
  float* sval = srec + SB * SRP;  // [NW][CW][2][64]
  int pkey = 0;
  float pw[12];
  float2 nv[CW], cv[CW];
  auto prefetch = [&](int k0, int n) {
    if (tid < n) {
      const SampleRec& r = rec[k0 + tid];
      pkey = r.key;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pw[q] = r.wx[q];
        pw[4 + q] = r.wy[q];
        pw[8 + q] = r.wz[q];
      }
    }
    const float2* vr = V + (long long)(it.voff + k0 - kbeg + lane) * cb + cg0 + q0;
#pragma unroll
    for (int q = 0; q < CW; ++q)
      nv[q] = (lane < n && q0 + q < cga) ? vr[q] : make_float2(0.f, 0.f);
  };
  if (kbeg < kend) prefetch(kbeg, min(SB, kend - kbeg));

  for (int k0 = kbeg; k0 < kend; k0 += SB) {
    const int n = min(SB, kend - k0);
    __syncthreads();  // previous batch consumed (and accumulator zeroed)
    if (tid < n) {
      float* d = srec + tid * SRP;
      d[0] = __int_as_float(pkey);
#pragma unroll
      for (int q = 0; q < 4; ++q) d[1 + q] = pw[q];
#pragma unroll
      for (int q = 0; q < 16; ++q) d[5 + q] = pw[4 + (q & 3)] * pw[8 + (q >> 2)];
    }
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      sval[((wave * CW + q) * 2) * 64 + lane] = nv[q].x;
      sval[((wave * CW + q) * 2 + 1) * 64 + lane] = nv[q].y;
    }
    if (tid < 64) {
      const int prev = __shfl_up(pkey, 1);
      const bool start = tid < n && pkey != (tid > 0 ? prev : rkey);
      const unsigned long long mask = __ballot(start);
      if (start) s_rs[__popcll(mask & ((1ull << tid) - 1ull))] = tid;
      if (tid == 0) {
        s_nr = __popcll(mask);
        s_sm[0] = (unsigned)mask;
        s_sm[1] = (unsigned)(mask >> 32);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CW; ++q)
      cv[q] = make_float2(sval[((wave * CW + q) * 2) * 64 + lane],
                          sval[((wave * CW + q) * 2 + 1) * 64 + lane]);
    if constexpr (VAR >= 2) {
      static_assert(SB == 64, "one run-start bit and one value lane per sample");
      // VAR 3: chunk c of 16 samples, sample 16 c + (lane & 15) in every row
      float2 cr[CW][4];
      if constexpr (VAR == 3) {
#pragma unroll
        for (int q = 0; q < CW; ++q)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            cr[q][c] = make_float2(sval[((wave * CW + q) * 2) * 64 + 16 * c + (lane & 15)],
                                   sval[((wave * CW + q) * 2 + 1) * 64 + 16 * c + (lane & 15)]);
      }
      const int vkey = __float_as_int(srec[lane * SRP]);
      const unsigned sm0 = __builtin_amdgcn_readfirstlane(s_sm[0]),
                     sm1 = __builtin_amdgcn_readfirstlane(s_sm[1]);
      if (k0 + SB < kend) prefetch(k0 + SB, min(SB, kend - k0 - SB));
      rw_batch<3, CW, VAR == 3>(lacc, srec, n, sm0, sm1, vkey, dx, dy, dz, active, cr, cv,
                                racc, rbase, rkey, rp);
      continue;
    }
    // lane j: key of sample j and start of run j of the batch (broadcast
    // by v_readlane below instead of a LDS round trip per run)
    const int vkey = __float_as_int(srec[lane * SRP]);
    const int vrs = s_rs[lane];
    if (k0 + SB < kend) prefetch(k0 + SB, min(SB, kend - k0 - SB));
    // one sample of the current run (uniform s: the lane reads are
    // broadcasts through scalar registers)
    auto one = [&](int s) {
      const float* d = srec + s * SRP;
      const float w = d[1 + dx] * d[5 + dy + 4 * dz];
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const float vr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv[q].x), s));
        const float vi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv[q].y), s));
        racc[q].x += w * vr;
        racc[q].y += w * vi;
      }
    };
    const int nr = active ? __builtin_amdgcn_readfirstlane(s_nr) : -1;
    int s = 0;
    for (int r = -1; r < nr; ++r) {
      const int s1 = (r + 1 < nr) ? __builtin_amdgcn_readlane(vrs, r + 1) : n;
      if (r >= 0) {
        if (rkey >= 0) {
#pragma unroll
          for (int q = 0; q < CW; ++q) {
            float* pl = acc + (size_t)(q0 + q) * 2 * H::PLANE + raddr;
            if constexpr (PF) {
              pl[0] = rbase[q].x + racc[q].x;
              pl[H::PLANE] = rbase[q].y + racc[q].y;
            } else {
              pl[0] += racc[q].x;
              pl[H::PLANE] += racc[q].y;
            }
            racc[q] = make_float2(0.f, 0.f);
          }
        }
        rkey = __builtin_amdgcn_readlane(vkey, s);
        raddr = __builtin_amdgcn_readfirstlane((rkey >> 16) * H::PZ + ((rkey >> 8) & 0xff) * H::PY +
                                               (rkey & 0xff)) + loff;
        if constexpr (PF) {
#pragma unroll
          for (int q = 0; q < CW; ++q) {
            const float* pl = acc + (size_t)(q0 + q) * 2 * H::PLANE + raddr;
            rbase[q] = make_float2(pl[0], pl[H::PLANE]);
          }
        }
      }
      // unrolled by hand (the broadcasts are convergent operations, which
      // the compiler does not unroll at a run-time trip count)
      if constexpr (PF) {
        for (; s + 8 <= s1; s += 8) {
          one(s);
          one(s + 1);
          one(s + 2);
          one(s + 3);
          one(s + 4);
          one(s + 5);
          one(s + 6);
          one(s + 7);
        }
      }
      for (; s + 4 <= s1; s += 4) {
        one(s);
        one(s + 1);
        one(s + 2);
        one(s + 3);
      }
      for (; s < s1; ++s) one(s);
    }
  }
  if (rkey >= 0) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      float* pl = VAR >= 2 ? rp + (size_t)q * 2 * H::PLANE
                           : acc + (size_t)(q0 + q) * 2 * H::PLANE + raddr;
      if constexpr (PF) {
        pl[0] = rbase[q].x + racc[q].x;
        pl[H::PLANE] = rbase[q].y + racc[q].y;
      } else {
        pl[0] += racc[q].x;
        pl[H::PLANE] += racc[q].y;
      }
    }
  }
  __syncthreads();
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
    int nty, int ntz, int mx, int my, int mz, float2* __restrict__ G, int xcd, int vec) {
  using H = Halo<NDIM>;
  constexpr int TV = H::TX * H::TY * H::TZ;
  constexpr int BPT = (TV + 255) / 256;  // blocks per tile
  constexpr int NGMAX = (kCoilChunk + CG - 1) / CG;
  const int b = xcd ? (int)xcd_contiguous(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int tile = b / BPT;
  const int v = (b - tile * BPT) * 256 + threadIdx.x;
  if (v >= TV) return;
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int gx = ix * H::TX + v % H::TX, gy = iy * H::TY + (v / H::TX) % H::TY,
            gz = iz * H::TZ + v / (H::TX * H::TY);
  if (gx >= mx || gy >= my || gz >= mz) return;
  // each cover as one word: (its share of the tile index) << 11 | (its share
  // of the offset in the halo'd tile); the shares of the three axes add up
  // without carries (tile index < 2^21, offset < 2^11)
  unsigned cx[6], cy[6], cz[6];
  int nx_, ny_, nz_ = 1;
  {
    int t[6], d[6];
    nx_ = halo_cover(gx, ix, ntx, H::TX, mx, t, d);
    for (int k = 0; k < nx_; ++k) cx[k] = ((unsigned)t[k] << 11) | (unsigned)d[k];
    ny_ = halo_cover(gy, iy, nty, H::TY, my, t, d);
    for (int k = 0; k < ny_; ++k)
      cy[k] = ((unsigned)(t[k] * ntx) << 11) | (unsigned)(d[k] * H::EX);
    cz[0] = 0;
    if (NDIM == 3) {
      nz_ = halo_cover(gz, iz, ntz, H::TZ, mz, t, d);
      for (int k = 0; k < nz_; ++k)
        cz[k] = ((unsigned)(t[k] * ntx * nty) << 11) | (unsigned)(d[k] * H::EX * H::EY);
    }
  }
  float2 acc[NGMAX * CG];
#pragma unroll
  for (int c = 0; c < NGMAX * CG; ++c) acc[c] = make_float2(0.f, 0.f);
  const size_t gstride = (size_t)H::EXT * CG;
  for (int a = 0; a < nz_; ++a)
    for (int b = 0; b < ny_; ++b)
      for (int d = 0; d < nx_; ++d) {
        const unsigned w = cz[a] + cy[b] + cx[d];
        const int t = (int)(w >> 11), e = (int)(w & 2047u);
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
  if (vec) {
    // even cb, 16-byte aligned G: coils two at a time
#pragma unroll
    for (int c = 0; c + 1 < NGMAX * CG; c += 2)
      if (c < cb)
        reinterpret_cast<float4*>(out)[c / 2] =
            make_float4(acc[c].x, acc[c].y, acc[c + 1].x, acc[c + 1].y);
  } else {
#pragma unroll
    for (int c = 0; c < NGMAX * CG; ++c)
      if (c < cb) out[c] = acc[c];
  }
}

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

template <int NDIM, int NW, int CW, bool SV = false, int VAR = 0>
int spread_items_launch(cs_ctx* c, int src, const float2* vals, int ldc, int c0, int cb,
                        int item0, int nitems) {
  using H = Halo<NDIM>;
  constexpr int CG = spread_cg<NDIM, NW, CW>();
  const int ng = (cb + CG - 1) / CG;
  if ((size_t)c->n_items * ng * H::EXT * CG > c->partial_elems)
    return fail(c, CS_EINVAL, "spread partial buffer too small");
  // the register-broadcast variant serves the 3D normal operator; 2D (four
  // coil slots per wave) and the caller's data use the LDS-staged one
  const bool rl = SV && NDIM == 3 && src == SRC_VALS;
  const size_t lds = rl ? sizeof(float) * ((size_t)CG * 2 * H::PLANE +
                                           kSpreadBatch * kSpreadRecPitch + CG * 2 * 64)
                        : spread_lds_bytes<NDIM, NW, CW>();
  if (lds > 160 * 1024) return fail(c, CS_EINVAL, "spread tile does not fit in LDS");
  if (nitems <= 0) return CS_OK;
  // shapes 9-12 (VAR 2, 3) take the register-weight loop in both kernels
  // (k_spread_items always with the DPP broadcasts)
  constexpr bool rw = VAR >= 2;
  auto kern = rl ? k_spread_rl<NW, CW, VAR>
                 : (src == SRC_VALS ? k_spread_items<NDIM, NW, CW, SRC_VALS, rw>
                                    : k_spread_items<NDIM, NW, CW, SRC_DATA, rw>);
  if (lds > 64 * 1024)
    CS_HIP(c, hipFuncSetAttribute((const void*)kern,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  CS_KLAUNCH(c, K_SPREAD, kern, item_group_grid(nitems, ng, c->grid_xcd), dim3(64 * NW), lds,
             c->stream, vals, ldc, c0, cb, c->rec, c->gitems, item0, c->ntile[2],
             c->ntile[1], c->partial, nitems, c->grid_xcd);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

template <int NDIM, int NW, int CW>
int merge_launch(cs_ctx* c, int cb, float2* grid) {
  using H = Halo<NDIM>;
  constexpr int CG = spread_cg<NDIM, NW, CW>();
  const int ng = (cb + CG - 1) / CG;
  constexpr long long TV = (long long)H::TX * H::TY * H::TZ;
  const long long blocks = c->ntiles * ((TV + 255) / 256);
  if (blocks > 0x7fffffffLL) return fail(c, CS_EINVAL, "spread merge grid too large");
  constexpr int NA = ((kCoilChunk + CG - 1) / CG) * CG;
  const int vec = c->grid_vec && cb % 2 == 0 && NA % 2 == 0 && ((uintptr_t)grid & 15) == 0;
  // the merge packs a cover's tile index and tile offset into one word
  if (c->ntiles >= (1LL << 21) || H::EXT >= 2048)
    return fail(c, CS_EINVAL, "spread merge: too many tiles");
  CS_KLAUNCH(c, K_MERGE, (k_spread_merge<NDIM, CG>), dim3((unsigned)blocks), dim3(256), 0,
             c->stream, c->partial, c->item_off, cb, ng, c->ntile[2], c->ntile[1],
             c->ntile[0], c->mx, c->my, c->mz, grid, c->merge_xcd, vec);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

// work-group shapes (waves NW, coils per lane CW); the coils of a group are
// NW * CW (3D) or 4 NW CW (2D, four coil slots of 16 taps per wave).
// `what`: 0 spread a range of items, 1 merge every slot into the grid.
template <int NDIM>
int spread_dispatch(cs_ctx* c, int what, int src, const float2* vals, int ldc, int c0, int cb,
                    int item0, int nitems, float2* grid) {
#define CS_SHAPE(NW, CW)                                                                   \
  return what == 0 ? spread_items_launch<NDIM, NW, CW>(c, src, vals, ldc, c0, cb, item0,  \
                                                       nitems)                             \
                   : merge_launch<NDIM, NW, CW>(c, cb, grid)
#define CS_SHAPE_SV(NW, CW, VAR)                                                           \
  return what == 0 ? spread_items_launch<NDIM, NW, CW, true, VAR>(c, src, vals, ldc, c0,  \
                                                                 cb, item0, nitems)        \
                   : merge_launch<NDIM, NW, CW>(c, cb, grid)
  switch (c->spread_cfg) {
    case 0: CS_SHAPE_SV(4, 1, 0);
    case 7: CS_SHAPE(4, 1);
    case 8: CS_SHAPE_SV(4, 1, 1);
    case 9: CS_SHAPE_SV(4, 1, 2);
    case 10: CS_SHAPE_SV(2, 2, 2);
    case 11: CS_SHAPE_SV(1, 4, 2);
    case 12: CS_SHAPE_SV(4, 1, 3);
    case 1: CS_SHAPE(2, 2);
    case 2: CS_SHAPE(2, 1);
    case 3: CS_SHAPE(1, 4);
    case 4: CS_SHAPE(4, 2);
    case 5: CS_SHAPE(1, 3);
    case 6:
      // all coils of the chunk in one work-group where the LDS allows (one
      // wave per coil), so every sample is staged once
      if constexpr (NDIM == 3) {
        if (cb <= 4) CS_SHAPE(4, 1);
        if (cb <= 6) CS_SHAPE(6, 1);
        if (cb <= 8) CS_SHAPE(8, 1);
        if (cb <= 12) CS_SHAPE(12, 1);
        CS_SHAPE(8, 1);
      } else {
        CS_SHAPE(4, 1);
      }
    default: CS_SHAPE_SV(4, 1, 0);
  }
#undef CS_SHAPE
#undef CS_SHAPE_SV
}

// largest coil-group size over the shapes above, for the partial buffer
int spread_max_group_elems(int ndim) {
  const int lpc = ndim == 3 ? 1 : 4;
  const int cgs[6] = {4 * lpc, 4 * lpc, 2 * lpc, 4 * lpc, 8 * lpc, 3 * lpc};
  int best = 0;
  for (int cg : cgs) best = std::max(best, ((kCoilChunk + cg - 1) / cg) * cg);
  return best;
}

int spread_items(cs_ctx* c, int src, const float2* vals, int ldc, int c0, int cb, int item0,
                 int nitems) {
  return c->ndim == 3
             ? spread_dispatch<3>(c, 0, src, vals, ldc, c0, cb, item0, nitems, nullptr)
             : spread_dispatch<2>(c, 0, src, vals, ldc, c0, cb, item0, nitems, nullptr);
}

int merge_slots(cs_ctx* c, int cb, float2* grid) {
  return c->ndim == 3 ? spread_dispatch<3>(c, 1, 0, nullptr, 0, 0, cb, 0, 0, grid)
                      : spread_dispatch<2>(c, 1, 0, nullptr, 0, 0, cb, 0, 0, grid);
}

int interp_items(cs_ctx* c, const float2* grid, int cb, int item0, int nitems, int wmode,
                 float2* out, int ldc, int c0, int caller_order) {
  return c->ndim == 3 ? interp_dispatch<3>(c, grid, cb, item0, nitems, wmode, out, ldc, c0,
                                           caller_order)
                      : interp_dispatch<2>(c, grid, cb, item0, nitems, wmode, out, ldc, c0,
                                           caller_order);
}

}  // namespace

int grid_normal(cs_ctx* c, const float2* grid, int cb, float2* out_grid) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "gridding coil chunk");
  for (size_t g = 0; g + 1 < c->group_off.size(); ++g) {
    const int i0 = c->group_off[g], i1 = c->group_off[g + 1];
    CS_TRY(interp_items(c, grid, cb, i0, i1 - i0, W_FULL, c->vbuf, cb, 0, 0));
    CS_TRY(spread_items(c, SRC_VALS, c->vbuf, cb, 0, cb, i0, i1 - i0));
  }
  return merge_slots(c, cb, out_grid);
}

int grid_interp(cs_ctx* c, const float2* grid, int cb, float2* y, int ldc, int c0) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "gridding coil chunk");
  return interp_items(c, grid, cb, 0, (int)c->n_items, W_SQRT, y, ldc, c0, 1);
}

int grid_spread_data(cs_ctx* c, const float2* y, int ldc, int c0, int cb, float2* out_grid) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "gridding coil chunk");
  CS_TRY(spread_items(c, SRC_DATA, y, ldc, c0, cb, 0, (int)c->n_items));
  return merge_slots(c, cb, out_grid);
}

namespace {

// ---- set-up of the trajectory on the GPU ------------------------------------

struct SetupGeom {
  int nd;
  int n[3], m[3], T[3], nt[3];  // image, grid, tile size, tiles per axis (z, y, x)
  double beta;
};

// One thread per sample (caller order): checks the coordinates and w, forms
// the record (first tap per axis relative to its tile, w, sqrt(w), caller
// index, kernel weights) and the sort key (tile, first tap in the tile) in
// the high 32 bits above the caller index, so that sorting the keys is a
// stable sort of the samples by tile and first tap.  err bit 1: a
// coordinate outside [-n/2, n/2); bit 2: w < 0 or NaN.
__global__ void k_setup_samples(const float* __restrict__ coords, const float* __restrict__ dcf,
                                long long N, SetupGeom g, SampleRec* __restrict__ rec,
                                unsigned long long* __restrict__ keys, int* __restrict__ err) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  SampleRec r{};
  int base[3] = {0, 0, 0};
  float* wts[3] = {r.wz, r.wy, r.wx};
  bool bad = false;
  for (int a = 3 - g.nd; a < 3; ++a) {
    const double k = coords[i * g.nd + (2 - a)];
    if (!(k >= -0.5 * g.n[a] && k < 0.5 * g.n[a])) {
      bad = true;
      continue;
    }
    const double u = k * (double)g.m[a] / (double)g.n[a];
    const double f = floor(u);
    const long long b = (long long)f - 1;
    for (int j = 0; j < 4; ++j) wts[a][j] = (float)kb_kernel(u - (double)(b + j), 4.0, g.beta);
    long long bw = b % g.m[a];
    if (bw < 0) bw += g.m[a];
    base[a] = (int)bw;
  }
  if (bad) atomicOr(err, 1);
  if (g.nd == 2) r.wz[0] = 1.f;
  const int lz = base[0] % g.T[0], ly = base[1] % g.T[1], lx = base[2] % g.T[2];
  r.key = lx | (ly << 8) | (lz << 16);
  r.orig = (int)i;
  const double w = dcf ? (double)dcf[i] : 1.0;
  if (!(w >= 0)) atomicOr(err, 2);
  r.w = (float)w;
  r.sw = (float)sqrt(w >= 0 ? w : 0.0);
  rec[i] = r;
  const unsigned long long t =
      ((unsigned long long)(base[0] / g.T[0]) * g.nt[1] + base[1] / g.T[1]) * g.nt[2] +
      base[2] / g.T[2];
  const unsigned long long tv = (unsigned long long)g.T[0] * g.T[1] * g.T[2];
  const unsigned long long k32 = t * tv + (unsigned long long)((lz * g.T[1] + ly) * g.T[2] + lx);
  keys[i] = (k32 << 32) | (unsigned long long)i;
}

__global__ void k_fill_keys(unsigned long long* keys, long long from, long long to) {
  const long long i = from + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) keys[i] = ~0ull;
}

// Bitonic sort of a power-of-two array of 64-bit keys, ascending.  Stage k
// merges runs of length k; step j compares elements j apart (direction by
// bit k of the index).  Steps with j >= 2048 run one pass over the array
// each; the steps j <= 1024 of a stage run in LDS, 2048 keys per block.
constexpr int kSortBlock = 2048;

__global__ __launch_bounds__(1024) void k_bitonic_local(unsigned long long* a, long long k0,
                                                        long long k1) {
  __shared__ unsigned long long s[kSortBlock];
  const long long base = (long long)blockIdx.x * kSortBlock;
  const int tid = threadIdx.x;
  s[tid] = a[base + tid];
  s[tid + 1024] = a[base + tid + 1024];
  __syncthreads();
  // stages k0 .. k1 (powers of two); for k > 2048 only its steps j <= 1024
  for (long long k = k0; k <= k1; k <<= 1) {
    for (int j = (int)(k / 2 < 1024 ? k / 2 : 1024); j > 0; j >>= 1) {
      const int i = 2 * tid - (tid & (j - 1));
      const bool asc = ((base + i) & k) == 0;
      const unsigned long long x = s[i], y = s[i + j];
      if ((x > y) == asc) {
        s[i] = y;
        s[i + j] = x;
      }
      __syncthreads();
    }
  }
  a[base + tid] = s[tid];
  a[base + tid + 1024] = s[tid + 1024];
}

__global__ void k_bitonic_global(unsigned long long* a, long long n, long long j, long long k) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n / 2) return;
  const long long i = 2 * t - (t & (j - 1));
  const bool asc = (i & k) == 0;
  const unsigned long long x = a[i], y = a[i + j];
  if ((x > y) == asc) {
    a[i] = y;
    a[i + j] = x;
  }
}

// sorted record j = record of the sample in the low half of sorted key j
__global__ void k_gather_sorted(const unsigned long long* __restrict__ keys,
                                const SampleRec* __restrict__ rec, long long N,
                                SampleRec* __restrict__ out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) out[j] = rec[keys[j] & 0xffffffffull];
}

// toff[t] = first sorted sample of tile t or later (lower bound of t * TV in
// the keys' high halves); toff[ntiles] = N
__global__ void k_tile_offsets(const unsigned long long* __restrict__ keys, long long N,
                               long long ntiles, unsigned long long tv, long long* toff) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  const unsigned long long want = (unsigned long long)t * tv;
  long long lo = 0, hi = N;
  while (lo < hi) {
    const long long mid = (lo + hi) / 2;
    if ((keys[mid] >> 32) < want) lo = mid + 1;
    else hi = mid;
  }
  toff[t] = lo;
}

unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int setup_noncart(cs_ctx* c, const float* coords_dev, const float* dcf_dev) {
  const long long N = c->N;
  const int nd = c->ndim;
  if (N > 0x7fffffffLL) return fail(c, CS_EINVAL, "more than 2^31 - 1 samples");
  if (N == 0) dcf_dev = nullptr;  // empty trajectory: the zero operator
  const int n[3] = {c->nz, c->ny, c->nx};
  const int m[3] = {c->mz, c->my, c->mx};

  // spread tiles: 8x8x8 (3D) or 16x16 (2D) voxels; the work-group shape is
  // a tuning knob (CS_SPREAD_CFG in the environment, see spread_dispatch)
  c->tile[0] = nd == 3 ? 8 : 1;
  c->tile[1] = nd == 3 ? 8 : 16;
  c->tile[2] = nd == 3 ? 8 : 16;
  for (int a = 3 - nd; a < 3; ++a)
    if (m[a] < 4) return fail(c, CS_EINVAL, "NUFFT grid shorter than the kernel");
  const char* cfg = std::getenv("CS_SPREAD_CFG");
  c->spread_cfg = cfg ? std::atoi(cfg) : kSpreadDefault;
  if (const char* e = std::getenv("CS_GRID_XCD")) c->grid_xcd = std::atoi(e) != 0;
  if (const char* e = std::getenv("CS_MERGE_XCD")) c->merge_xcd = std::atoi(e) != 0;
  const char* icfg = std::getenv("CS_INTERP_CFG");
  c->interp_cfg = icfg ? std::atoi(icfg) : 3;
  // samples per item group of the normal operator (CS_GROUP_SAMPLES in the
  // environment; at least one work item)
  const char* gcfg = std::getenv("CS_GROUP_SAMPLES");
  long long group_cap = gcfg ? std::atoll(gcfg) : kGroupSamples;
  group_cap = std::max(group_cap, 2048LL);
  for (int a = 0; a < 3; ++a) c->ntile[a] = (m[a] + c->tile[a] - 1) / c->tile[a];
  c->ntiles = (long long)c->ntile[0] * c->ntile[1] * c->ntile[2];
  const unsigned long long tv = (unsigned long long)c->tile[0] * c->tile[1] * c->tile[2];
  if ((unsigned long long)c->ntiles * tv >= (1ull << 32))
    return fail(c, CS_EUNSUPPORTED, "NUFFT grid too large for the 32-bit sort keys");

  // records, keys, bitonic sort (the key's low half, the caller index, makes
  // it stable), sorted records and tile offsets, all on the GPU
  CS_HIP(c, hipMalloc(&c->rec, sizeof(SampleRec) * std::max(1LL, N)));
  std::vector<long long> toff(c->ntiles + 1, 0);
  if (N > 0) {
    long long np = kSortBlock;
    while (np < N) np *= 2;
    SampleRec* rec_in = nullptr;
    unsigned long long* keys = nullptr;
    long long* toff_dev = nullptr;
    int* err_dev = nullptr;
    auto release = [&]() {
      if (rec_in) (void)hipFree(rec_in);
      if (keys) (void)hipFree(keys);
      if (toff_dev) (void)hipFree(toff_dev);
      if (err_dev) (void)hipFree(err_dev);
    };
    auto run = [&]() -> int {
      CS_HIP(c, hipMalloc(&rec_in, sizeof(SampleRec) * N));
      CS_HIP(c, hipMalloc(&keys, sizeof(unsigned long long) * np));
      CS_HIP(c, hipMalloc(&toff_dev, sizeof(long long) * (c->ntiles + 1)));
      CS_HIP(c, hipMalloc(&err_dev, sizeof(int)));
      CS_HIP(c, hipMemsetAsync(err_dev, 0, sizeof(int), c->stream));
      SetupGeom g{};
      g.nd = nd;
      for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.m[a] = m[a];
        g.T[a] = c->tile[a];
        g.nt[a] = c->ntile[a];
      }
      g.beta = c->beta;
      hipLaunchKernelGGL(k_setup_samples, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream,
                         coords_dev, dcf_dev, N, g, rec_in, keys, err_dev);
      if (np > N)
        hipLaunchKernelGGL(k_fill_keys, dim3(blocks_for(np - N, 256)), dim3(256), 0, c->stream,
                           keys, N, np);
      const unsigned nb = (unsigned)(np / kSortBlock);
      hipLaunchKernelGGL(k_bitonic_local, dim3(nb), dim3(1024), 0, c->stream, keys, 2LL,
                         (long long)kSortBlock);
      for (long long k = 2 * kSortBlock; k <= np; k *= 2) {
        for (long long j = k / 2; j >= kSortBlock; j /= 2)
          hipLaunchKernelGGL(k_bitonic_global, dim3(blocks_for(np / 2, 256)), dim3(256), 0,
                             c->stream, keys, np, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3(nb), dim3(1024), 0, c->stream, keys, k, k);
      }
      CS_HIP(c, hipGetLastError());
      hipLaunchKernelGGL(k_gather_sorted, dim3(blocks_for(N, 256)), dim3(256), 0, c->stream,
                         keys, rec_in, N, c->rec);
      hipLaunchKernelGGL(k_tile_offsets, dim3(blocks_for(c->ntiles + 1, 256)), dim3(256), 0,
                         c->stream, keys, N, c->ntiles, tv, toff_dev);
      CS_HIP(c, hipGetLastError());
      int err = 0;
      CS_HIP(c, hipMemcpyAsync(&err, err_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      CS_HIP(c, hipMemcpyAsync(toff.data(), toff_dev, sizeof(long long) * (c->ntiles + 1),
                               hipMemcpyDeviceToHost, c->stream));
      CS_HIP(c, hipStreamSynchronize(c->stream));
      if (err & 1) return fail(c, CS_EINVAL, "coordinate outside [-n/2, n/2)");
      if (err & 2) return fail(c, CS_EINVAL, "density compensation must be >= 0");
      return CS_OK;
    };
    const int rc = run();
    release();
    if (rc != CS_OK) return rc;
  }
  if (dcf_dev) {
    CS_HIP(c, hipMalloc(&c->dcf_orig, sizeof(float) * N));
    CS_HIP(c, hipMemcpyAsync(c->dcf_orig, dcf_dev, sizeof(float) * N, hipMemcpyDeviceToDevice,
                             c->stream));
  }

  // work items: each tile's samples in chunks of at most `chunk` (2048 in 3D;
  // 512 in 2D, where a slice has few tiles and the heaviest items set the
  // launch time); the slot of an item is its index in tile order, so the
  // slots of tile t are item_off[t] .. item_off[t + 1]
  long long chunk = nd == 3 ? 2048 : 512;
  if (const char* e = std::getenv("CS_ITEM_SAMPLES")) chunk = std::max(64LL, std::atoll(e));
  std::vector<GridItem> items;
  std::vector<int> ioff(c->ntiles + 1, 0);
  for (long long t = 0; t < c->ntiles; ++t) {
    for (long long k = toff[t]; k < toff[t + 1]; k += chunk) {
      GridItem g{};
      g.tile = (int)t;
      g.kbeg = (int)k;
      g.kend = (int)std::min(toff[t + 1], k + chunk);
      g.slot = (int)items.size();
      items.push_back(g);
    }
    ioff[t + 1] = (int)items.size();
  }
  // item groups of the normal operator: at most group_cap samples each,
  // whose values (one row of <= kCoilChunk coils per sample) go to the value
  // buffer at the item's offset voff.  Items are dealt, heaviest first,
  // round-robin to the groups, and each group runs its heaviest items first
  // so that the long ones start early.
  std::stable_sort(items.begin(), items.end(), [](const GridItem& a, const GridItem& b) {
    return (a.kend - a.kbeg) > (b.kend - b.kbeg);
  });
  const long long ngroups = std::max(1LL, (N + group_cap - 1) / group_cap);
  std::vector<std::vector<GridItem>> groups(ngroups);
  std::vector<long long> gsize(ngroups, 0);
  for (const GridItem& it : items) {
    // the lightest group that still has room (dealing in order keeps them level)
    long long best = -1;
    for (long long g = 0; g < ngroups; ++g)
      if (gsize[g] + (it.kend - it.kbeg) <= group_cap && (best < 0 || gsize[g] < gsize[best]))
        best = g;
    if (best < 0) {
      best = (long long)groups.size();
      groups.emplace_back();
      gsize.push_back(0);
    }
    GridItem g = it;
    g.voff = (int)gsize[best];
    gsize[best] += it.kend - it.kbeg;
    groups[best].push_back(g);
  }
  std::vector<GridItem> ordered;
  c->group_off.assign(1, 0);
  for (auto& g : groups) {
    if (g.empty()) continue;
    ordered.insert(ordered.end(), g.begin(), g.end());
    c->group_off.push_back((int)ordered.size());
  }
  c->n_items = (long long)ordered.size();
  CS_HIP(c, hipMalloc(&c->gitems, sizeof(GridItem) * std::max<size_t>(1, ordered.size())));
  if (!ordered.empty())
    CS_HIP(c, hipMemcpy(c->gitems, ordered.data(), sizeof(GridItem) * ordered.size(),
                        hipMemcpyHostToDevice));
  CS_HIP(c, hipMalloc(&c->item_off, sizeof(int) * ioff.size()));
  CS_HIP(c, hipMemcpy(c->item_off, ioff.data(), sizeof(int) * ioff.size(),
                      hipMemcpyHostToDevice));
  const size_t ext = nd == 3 ? (size_t)Halo<3>::EXT : (size_t)Halo<2>::EXT;
  c->partial_elems = std::max<size_t>(1, (size_t)c->n_items * ext * spread_max_group_elems(nd));
  CS_HIP(c, hipMalloc(&c->partial, sizeof(float2) * c->partial_elems));
  // values of the largest item group, kCoilChunk coils per sample
  long long gmax = 1;
  for (long long g : gsize) gmax = std::max(gmax, g);
  // padded by kCoilChunk coils: the scalar-value spreading reads whole runs
  // of a wave's coils, which run past the last row when a chunk is partial
  c->vbuf_pad = kCoilChunk;
  CS_HIP(c, hipMalloc(&c->vbuf, sizeof(float2) * ((size_t)gmax * kCoilChunk + kCoilChunk)));
  return CS_OK;
}

}  // namespace cs
