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
#pragma unroll
  for (int dz = 0; dz < nzt; ++dz) {
    int z = r.bz + dz;
    if (z >= mz) z -= mz;
    const float wz = NDIM == 3 ? r.wz[dz] : 1.f;
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
      int y = r.by + dy;
      if (y >= my) y -= my;
      const float wyz = wz * r.wy[dy];
      const long long row = ((long long)z * my + y) * mx;
#pragma unroll
      for (int dx = 0; dx < 4; ++dx) {
        const float w = wyz * r.wx[dx];
        const float2* p = G + (row + xs[dx]) * cb;
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

template <int NDIM>
__global__ __launch_bounds__(64) void k_spread(const float2* __restrict__ V, int cb,
                                               const SampleRec* __restrict__ rec,
                                               const int* __restrict__ tile_off,
                                               const int* __restrict__ tile_list,
                                               int tx, int ty, int tz, int ntx, int nty,
                                               int mx, int my, int mz,
                                               float2* __restrict__ G) {
  extern __shared__ float lds[];
  const int tile = blockIdx.x;
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int x0 = ix * tx, y0 = iy * ty, z0 = iz * tz;
  const int ex = min(tx, mx - x0), ey = min(ty, my - y0), ez = min(tz, mz - z0);
  const int nvox = tx * ty * tz;
  const int lane = threadIdx.x;
  for (int i = lane; i < nvox * cb * 2; i += 64) lds[i] = 0.f;
  __syncthreads();

  const int dx = lane & 3, dy = (lane >> 2) & 3, dz = lane >> 4;
  const bool lane_ok = NDIM == 3 || dz == 0;
  const int kbeg = tile_off[tile], kend = tile_off[tile + 1];
  for (int k = kbeg; k < kend; ++k) {
    const int j = tile_list[k];
    const SampleRec& r = rec[j];
    int gx = r.bx + dx;
    if (gx >= mx) gx -= mx;
    int gy = r.by + dy;
    if (gy >= my) gy -= my;
    int gz = NDIM == 3 ? r.bz + dz : 0;
    if (gz >= mz) gz -= mz;
    const int lx = gx - x0, ly = gy - y0, lz = gz - z0;
    const bool in = lane_ok && (unsigned)lx < (unsigned)ex && (unsigned)ly < (unsigned)ey &&
                    (unsigned)lz < (unsigned)ez;
    if (in) {
      float w = sel4(r.wx, dx) * sel4(r.wy, dy);
      if (NDIM == 3) w *= sel4(r.wz, dz);
      const int e = ((lz * ty + ly) * tx + lx) * cb;
      const float2* v = V + (long long)j * cb;
      for (int c = 0; c < cb; ++c) {
        const float2 val = v[c];
        atomicAdd(&lds[2 * (e + c)], w * val.x);
        atomicAdd(&lds[2 * (e + c) + 1], w * val.y);
      }
    }
  }
  __syncthreads();
  const int nout = ex * ey * ez * cb;
  for (int i = lane; i < nout; i += 64) {
    const int c = i % cb;
    const int v = i / cb;
    const int lx = v % ex, ly = (v / ex) % ey, lz = v / (ex * ey);
    const int e = ((lz * ty + ly) * tx + lx) * cb + c;
    const long long gidx =
        (((long long)(z0 + lz) * my + (y0 + ly)) * mx + (x0 + lx)) * cb + c;
    G[gidx] = make_float2(lds[2 * e], lds[2 * e + 1]);
  }
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
  if (cb <= 2) CS_INTERP(2);
  else if (cb <= 4) CS_INTERP(4);
  else if (cb <= 8) CS_INTERP(8);
  else if (cb <= 12) CS_INTERP(12);
  else CS_INTERP(16);
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

int launch_spread(cs_ctx* c, const float2* vals, int cb, float2* grid) {
  if (cb < 1 || cb > kCoilChunk) return fail(c, CS_EINVAL, "spread coil chunk");
  const int tz = c->tile[0], ty = c->tile[1], tx = c->tile[2];
  const size_t lds = sizeof(float) * 2 * (size_t)tx * ty * tz * cb;
  if (lds > 160 * 1024) return fail(c, CS_EINVAL, "spread tile does not fit in LDS");
  const unsigned nb = (unsigned)c->ntiles;
  if (c->ndim == 3)
    CS_KLAUNCH(c, K_SPREAD, k_spread<3>, dim3(nb), dim3(64), lds, c->stream, vals, cb, c->rec,
                       c->tile_off, c->tile_list, tx, ty, tz, c->ntile[2], c->ntile[1],
                       c->mx, c->my, c->mz, grid);
  else
    CS_KLAUNCH(c, K_SPREAD, k_spread<2>, dim3(nb), dim3(64), lds, c->stream, vals, cb, c->rec,
                       c->tile_off, c->tile_list, tx, ty, tz, c->ntile[2], c->ntile[1],
                       c->mx, c->my, c->mz, grid);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
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
    c->tile[0] = 8; c->tile[1] = 8; c->tile[2] = 8;
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
  return CS_OK;
}

}  // namespace cs
