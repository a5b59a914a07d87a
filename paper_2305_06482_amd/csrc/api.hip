// C ABI of the coil-sketching library: contexts, the SENSE operator and its
// adjoint / normal operator (Sec. 2.1, Eqs. 1-2, 5), the structured sketch
// (Sec. 2.3.2-2.3.3, Eqs. 11-13) and Algorithm 1 with FISTA inner solves
// (Sec. 2.3.4, Sec. 3.3.1).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>

#include "cs_internal.h"

namespace {
std::string g_create_error;

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output number n from state
// seed is mix(seed + n * 0x9E3779B97F4A7C15).
uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Rademacher block of outer iteration t: entry (a, b) is -1 when the top bit
// of output number ((t << 32) | (a * cols + b)) + 1 is set, else +1.
void rademacher(uint64_t seed, int t, int S, int cols, std::vector<int8_t>& out) {
  out.resize((size_t)S * cols);
  for (int a = 0; a < S; ++a)
    for (int b = 0; b < cols; ++b) {
      const uint64_t ctr = ((uint64_t)(uint32_t)t << 32) | (uint64_t)(a * cols + b);
      const uint64_t z = splitmix64_mix(seed + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
      out[(size_t)a * cols + b] = (z >> 63) ? -1 : 1;
    }
}

// Gaussian block of outer iteration t (unit variance): entry e = a cols + b
// takes outputs c + 1 and c + 2, c = (t << 32) | 2e, as uniforms
// u1 in (0, 1] and u2 in [0, 1), and the Box-Muller value
// sqrt(-2 ln u1) cos(2 pi u2).
void gaussian(uint64_t seed, int t, int S, int cols, std::vector<double>& out) {
  out.resize((size_t)S * cols);
  for (int a = 0; a < S; ++a)
    for (int b = 0; b < cols; ++b) {
      const uint64_t e = (uint64_t)(a * cols + b);
      const uint64_t ctr = ((uint64_t)(uint32_t)t << 32) | (2 * e);
      const uint64_t z1 = splitmix64_mix(seed + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
      const uint64_t z2 = splitmix64_mix(seed + (ctr + 2) * 0x9E3779B97F4A7C15ULL);
      const double u1 = (double)((z1 >> 11) + 1) * 0x1.0p-53;
      const double u2 = (double)(z2 >> 11) * 0x1.0p-53;
      out[(size_t)e] = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    }
}
}  // namespace

namespace cs {

int fail(cs_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

namespace {
hipEvent_t pool_event(cs_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

void prof_begin(cs_ctx* c, int kind) {
  if (!c->prof) return;
  cs_ctx::ProfRec r{kind, pool_event(c), pool_event(c)};
  if (!r.a || !r.b) return;
  (void)hipEventRecord(r.a, c->stream);
  c->prof_recs.push_back(r);
}

void prof_end(cs_ctx* c) {
  if (!c->prof || c->prof_recs.empty()) return;
  (void)hipEventRecord(c->prof_recs.back().b, c->stream);
}

namespace {

PassArgs blank(int cb) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.cb = cb;
  a.src_ldc = cb;
  a.dst_ldc = cb;
  return a;
}

int with_plan(cs_ctx* c, PassArgs& a, int L) {
  const FFTPlan* p = nullptr;
  CS_TRY(get_plan(c, L, &p));
  fill_plan(a, p);
  return CS_OK;
}

// ---- Cartesian (2D): F~ = U F~_u, unitary FFT, zero-filled data -----------

// y pass from the image: x * maps / sqrt(D) -> FFT_y -> grid [ny][nx][cb]
// (or, with a ky-only mask, the whole normal operator in one pass)
int cart_first(cs_ctx* c, const float2* x, const float2* maps, int ldc, int c0, int cb,
               float2* dst, bool fused_normal, float2* out) {
  PassArgs a = blank(cb);
  CS_TRY(with_plan(c, a, c->ny));
  a.n_in = a.n_out = c->ny;
  a.dir = -1;
  a.inner = (long long)c->nx * cb;
  a.prologue = PRO_IMAGE;
  a.img = x;
  a.maps = maps;
  a.maps_ldc = ldc;
  a.maps_c0 = c0;
  a.P = c->nx;
  a.da = c->da[1];
  a.dp = c->dp_y;
  if (fused_normal) {
    // F_x^H F_x = I: only the unitary y transform pair remains
    a.da = c->da_y1d;
    a.mid = MID_MASK_IFFT;
    a.mask = c->mask;
    a.mask_os = 0;
    a.mask_rs = c->nx;
    a.epilogue = EPI_IMAGE;
    a.img_out = out;
    a.accumulate = c0 > 0;
  } else {
    a.dst = dst;
    a.dst_rs = (long long)c->nx * cb;
  }
  return launch_pass(c, a, 1);
}

// y pass to the image: IFFT_y -> conj(maps) sum / sqrt(D)
int cart_last(cs_ctx* c, const float2* src, const float2* maps, int ldc, int c0, int cb,
              float2* out) {
  PassArgs a = blank(cb);
  CS_TRY(with_plan(c, a, c->ny));
  a.n_in = a.n_out = c->ny;
  a.dir = +1;
  a.inner = (long long)c->nx * cb;
  a.src = src;
  a.src_rs = (long long)c->nx * cb;
  a.epilogue = EPI_IMAGE;
  a.img_out = out;
  a.accumulate = c0 > 0;
  a.maps = maps;
  a.maps_ldc = ldc;
  a.maps_c0 = c0;
  a.P = c->nx;
  a.da = c->da[1];
  a.dp = c->dp_y;
  return launch_pass(c, a, 1);
}

// x pass over rows ky: mode 0 = FFT, mask, IFFT (normal); 1 = FFT, mask -> y;
// 2 = mask y, IFFT (adjoint)
int cart_xpass(cs_ctx* c, int mode, const float2* src, long long src_os, long long src_rs,
               int src_ldc, int src_c0, float2* dst, long long dst_os, long long dst_rs,
               int dst_ldc, int dst_c0, int cb) {
  PassArgs a = blank(cb);
  CS_TRY(with_plan(c, a, c->nx));
  a.n_in = a.n_out = c->nx;
  a.inner = cb;
  a.src = src; a.src_os = src_os; a.src_rs = src_rs; a.src_ldc = src_ldc; a.src_c0 = src_c0;
  a.dst = dst; a.dst_os = dst_os; a.dst_rs = dst_rs; a.dst_ldc = dst_ldc; a.dst_c0 = dst_c0;
  a.mask = c->mask;
  a.mask_os = c->nx;
  a.mask_rs = 1;
  if (mode == 0) { a.dir = -1; a.mid = MID_MASK_IFFT; }
  if (mode == 1) { a.dir = -1; a.mid = MID_MASK; }
  if (mode == 2) { a.dir = +1; a.premask = 1; }
  return launch_pass(c, a, c->ny);
}

int cart_normal(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* x,
                float2* out) {
  if (c->mask1d) return cart_first(c, x, maps, ldc, c0, cb, nullptr, true, out);
  const long long row = (long long)c->nx * cb;
  CS_TRY(cart_first(c, x, maps, ldc, c0, cb, c->gridA, false, nullptr));
  CS_TRY(cart_xpass(c, 0, c->gridA, row, cb, cb, 0, c->gridA, row, cb, cb, 0, cb));
  return cart_last(c, c->gridA, maps, ldc, c0, cb, out);
}

int cart_apply(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* x,
               float2* y) {
  const long long row = (long long)c->nx * cb;
  CS_TRY(cart_first(c, x, maps, ldc, c0, cb, c->gridA, false, nullptr));
  return cart_xpass(c, 1, c->gridA, row, cb, cb, 0, y, (long long)c->nx * ldc, ldc, ldc, c0,
                    cb);
}

int cart_adjoint(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* y,
                 float2* out) {
  const long long row = (long long)c->nx * cb;
  CS_TRY(cart_xpass(c, 2, y, (long long)c->nx * ldc, ldc, ldc, c0, c->gridA, row, cb, cb, 0,
                    cb));
  return cart_last(c, c->gridA, maps, ldc, c0, cb, out);
}

// ---- non-Cartesian: deapodise, zero-pad, FFT on the sigma-grid, KB gridding --

// forward passes image -> oversampled grid [mz][my][mx][cb]; returns the buffer
int nc_forward(cs_ctx* c, const float2* x, const float2* maps, int ldc, int c0, int cb,
               float2** result) {
  const int nz = c->nz, ny = c->ny, nx = c->nx, mz = c->mz, my = c->my, mx = c->mx;
  float2* A = c->gridA;
  float2* B = c->gridB;
  if (c->ndim == 3) {
    PassArgs a = blank(cb);  // z
    CS_TRY(with_plan(c, a, mz));
    a.n_in = nz; a.pad_in = 1; a.n_out = mz; a.dir = -1;
    a.inner = (long long)ny * nx * cb;
    a.prologue = PRO_IMAGE; a.img = x; a.maps = maps; a.maps_ldc = ldc; a.maps_c0 = c0;
    a.P = (long long)ny * nx; a.da = c->da[0]; a.dp = c->dp_z;
    a.dst = A; a.dst_rs = (long long)ny * nx * cb;
    CS_TRY(launch_pass(c, a, 1));
    PassArgs b = blank(cb);  // y
    CS_TRY(with_plan(c, b, my));
    b.n_in = ny; b.pad_in = 1; b.n_out = my; b.dir = -1;
    b.inner = (long long)nx * cb;
    b.src = A; b.src_os = (long long)ny * nx * cb; b.src_rs = (long long)nx * cb;
    b.dst = B; b.dst_os = (long long)my * nx * cb; b.dst_rs = (long long)nx * cb;
    CS_TRY(launch_pass(c, b, mz));
    PassArgs d = blank(cb);  // x
    CS_TRY(with_plan(c, d, mx));
    d.n_in = nx; d.pad_in = 1; d.n_out = mx; d.dir = -1;
    d.inner = cb;
    d.src = B; d.src_os = (long long)nx * cb; d.src_rs = cb;
    d.dst = A; d.dst_os = (long long)mx * cb; d.dst_rs = cb;
    CS_TRY(launch_pass(c, d, (long long)mz * my));
    *result = A;
  } else {
    PassArgs a = blank(cb);  // y
    CS_TRY(with_plan(c, a, my));
    a.n_in = ny; a.pad_in = 1; a.n_out = my; a.dir = -1;
    a.inner = (long long)nx * cb;
    a.prologue = PRO_IMAGE; a.img = x; a.maps = maps; a.maps_ldc = ldc; a.maps_c0 = c0;
    a.P = nx; a.da = c->da[1]; a.dp = c->dp_y;
    a.dst = A; a.dst_rs = (long long)nx * cb;
    CS_TRY(launch_pass(c, a, 1));
    PassArgs d = blank(cb);  // x
    CS_TRY(with_plan(c, d, mx));
    d.n_in = nx; d.pad_in = 1; d.n_out = mx; d.dir = -1;
    d.inner = cb;
    d.src = A; d.src_os = (long long)nx * cb; d.src_rs = cb;
    d.dst = B; d.dst_os = (long long)mx * cb; d.dst_rs = cb;
    CS_TRY(launch_pass(c, d, my));
    *result = B;
  }
  return CS_OK;
}

// adjoint passes grid G [mz][my][mx][cb] -> image (conj-map coil sum); `tmp`
// is the other grid buffer; G is overwritten
int nc_adjoint_grid(cs_ctx* c, float2* G, float2* tmp, const float2* maps, int ldc, int c0,
                    int cb, float2* out) {
  const int nz = c->nz, ny = c->ny, nx = c->nx, mz = c->mz, my = c->my, mx = c->mx;
  PassArgs d = blank(cb);  // x
  CS_TRY(with_plan(c, d, mx));
  d.n_in = mx; d.n_out = nx; d.pad_out = 1; d.dir = +1;
  d.inner = cb;
  d.src = G; d.src_os = (long long)mx * cb; d.src_rs = cb;
  d.dst = tmp; d.dst_os = (long long)nx * cb; d.dst_rs = cb;
  CS_TRY(launch_pass(c, d, (long long)mz * my));
  if (c->ndim == 3) {
    PassArgs b = blank(cb);  // y
    CS_TRY(with_plan(c, b, my));
    b.n_in = my; b.n_out = ny; b.pad_out = 1; b.dir = +1;
    b.inner = (long long)nx * cb;
    b.src = tmp; b.src_os = (long long)my * nx * cb; b.src_rs = (long long)nx * cb;
    b.dst = G; b.dst_os = (long long)ny * nx * cb; b.dst_rs = (long long)nx * cb;
    CS_TRY(launch_pass(c, b, mz));
    PassArgs a = blank(cb);  // z
    CS_TRY(with_plan(c, a, mz));
    a.n_in = mz; a.n_out = nz; a.pad_out = 1; a.dir = +1;
    a.inner = (long long)ny * nx * cb;
    a.src = G; a.src_rs = (long long)ny * nx * cb;
    a.epilogue = EPI_IMAGE; a.img_out = out; a.accumulate = c0 > 0;
    a.maps = maps; a.maps_ldc = ldc; a.maps_c0 = c0;
    a.P = (long long)ny * nx; a.da = c->da[0]; a.dp = c->dp_z;
    return launch_pass(c, a, 1);
  }
  PassArgs a = blank(cb);  // y
  CS_TRY(with_plan(c, a, my));
  a.n_in = my; a.n_out = ny; a.pad_out = 1; a.dir = +1;
  a.inner = (long long)nx * cb;
  a.src = tmp; a.src_rs = (long long)nx * cb;
  a.epilogue = EPI_IMAGE; a.img_out = out; a.accumulate = c0 > 0;
  a.maps = maps; a.maps_ldc = ldc; a.maps_c0 = c0;
  a.P = nx; a.da = c->da[1]; a.dp = c->dp_y;
  return launch_pass(c, a, 1);
}

int nc_normal(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* x,
              float2* out) {
  float2* G = nullptr;
  CS_TRY(nc_forward(c, x, maps, ldc, c0, cb, &G));
  float2* other = G == c->gridA ? c->gridB : c->gridA;
  CS_TRY(grid_normal(c, G, cb, other));
  return nc_adjoint_grid(c, other, G, maps, ldc, c0, cb, out);
}

int nc_apply(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* x,
             float2* y) {
  float2* G = nullptr;
  CS_TRY(nc_forward(c, x, maps, ldc, c0, cb, &G));
  return grid_interp(c, G, cb, y, ldc, c0);
}

int nc_adjoint(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* y,
               float2* out) {
  CS_TRY(grid_spread_data(c, y, ldc, c0, cb, c->gridA));
  return nc_adjoint_grid(c, c->gridA, c->gridB, maps, ldc, c0, cb, out);
}

// data_arg: which of a (1) or b (2) is sample data, which may be NULL for an
// empty trajectory (0: both are images)
int check_ready(cs_ctx* c, const void* maps, int ncoil, const void* a, const void* b,
                int data_arg = 0) {
  if (!c) return CS_EINVAL;
  if (!c->have_op) return fail(c, CS_EINVAL, "cs_set_operator has not been called");
  const bool empty = c->g.kind == CS_NONCART && c->N == 0;
  if (!maps || (!a && !(empty && data_arg == 1)) || (!b && !(empty && data_arg == 2)))
    return fail(c, CS_EINVAL, "null pointer");
  if (ncoil < 1 || ncoil > 64) return fail(c, CS_EINVAL, "ncoil must be in [1, 64]");
  return CS_OK;
}

int chunk_loop(cs_ctx* c, int ncoil,
               int (*fn)(cs_ctx*, const float2*, int, int, int, const float2*, float2*),
               const float2* maps, const float2* in, float2* out) {
  const int chunk = c->g.kind == CS_NONCART ? kCoilChunk : kCoilChunk;
  for (int c0 = 0; c0 < ncoil; c0 += chunk) {
    const int cb = std::min(chunk, ncoil - c0);
    CS_TRY(fn(c, maps, ncoil, c0, cb, in, out));
  }
  return CS_OK;
}

int op_apply(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* x,
             float2* y) {
  return c->g.kind == CS_CART ? cart_apply(c, maps, ldc, c0, cb, x, y)
                              : nc_apply(c, maps, ldc, c0, cb, x, y);
}
int op_adjoint(cs_ctx* c, const float2* maps, int ldc, int c0, int cb, const float2* y,
               float2* x) {
  return c->g.kind == CS_CART ? cart_adjoint(c, maps, ldc, c0, cb, y, x)
                              : nc_adjoint(c, maps, ldc, c0, cb, y, x);
}
int op_normal_chunk(cs_ctx* c, const float2* maps, int ldc, int c0, int cb,
                    const float2* x, float2* out) {
  return c->g.kind == CS_CART ? cart_normal(c, maps, ldc, c0, cb, x, out)
                              : nc_normal(c, maps, ldc, c0, cb, x, out);
}

int upload_table(cs_ctx* c, float** dst, const std::vector<float>& v) {
  CS_HIP(c, hipMalloc(dst, sizeof(float) * std::max<size_t>(1, v.size())));
  CS_HIP(c, hipMemcpy(*dst, v.data(), sizeof(float) * v.size(), hipMemcpyHostToDevice));
  return CS_OK;
}

// FFT plans (twiddle tables) of every transform length the operator uses,
// made here so that no operator call allocates.  A length with a prime
// factor other than 2, 3, 5 gets no plan: the context still serves the
// building blocks, and every FFT on that length fails with CS_EINVAL (before
// any allocation).
int create_plans(cs_ctx* c) {
  std::vector<int> Ls;
  if (c->g.kind == CS_CART) {
    Ls = {c->ny, c->nx};
  } else {
    Ls = {c->my, c->mx};
    if (c->ndim == 3) Ls.push_back(c->mz);
  }
  for (int L : Ls) {
    int n = L;
    for (int f : {2, 3, 5})
      while (n % f == 0) n /= f;
    const FFTPlan* p = nullptr;
    if (n == 1) CS_TRY(get_plan(c, L, &p));
  }
  return CS_OK;
}

// Geometry checks and the derived sizes (no device work).
int init_geometry(cs_ctx* c, const cs_geom* g) {
  if (g->ndim != 2 && g->ndim != 3) return fail(nullptr, CS_EINVAL, "ndim must be 2 or 3");
  if (g->ncoil < 1 || g->ncoil > 64) return fail(nullptr, CS_EINVAL, "ncoil must be in [1, 64]");
  if (g->kind != CS_CART && g->kind != CS_NONCART) return fail(nullptr, CS_EINVAL, "kind");
  if (g->kind == CS_CART && g->ndim != 2)
    return fail(nullptr, CS_EUNSUPPORTED, "Cartesian operator is 2D only");
  for (int a = 0; a < g->ndim; ++a)
    if (g->n[a] < 4 || g->n[a] > kMaxFFT) return fail(nullptr, CS_EINVAL, "image size");
  if (g->kind == CS_NONCART) {
    if (g->kwidth != 4) return fail(nullptr, CS_EUNSUPPORTED, "only kernel width 4");
    if (!(g->sigma >= 1.0f && g->sigma <= 3.0f)) return fail(nullptr, CS_EINVAL, "sigma");
    if (g->nsamp < 0 || g->nsamp > 0x7fffffffLL) return fail(nullptr, CS_EINVAL, "nsamp");
  }
  if (g->wav_levels < 0 || g->wav_levels > 10) return fail(nullptr, CS_EINVAL, "wav_levels");
  for (int a = 0; a < g->ndim; ++a)
    if (g->n[a] % (1 << g->wav_levels) != 0)
      return fail(nullptr, CS_EINVAL, "image size not divisible by 2^wav_levels");
  c->g = *g;
  c->ndim = g->ndim;
  c->C = g->ncoil;
  if (g->ndim == 3) {
    c->nz = g->n[0]; c->ny = g->n[1]; c->nx = g->n[2];
  } else {
    c->nz = 1; c->ny = g->n[0]; c->nx = g->n[1];
  }
  c->D = (long long)c->nz * c->ny * c->nx;
  if (g->kind == CS_NONCART) {
    auto m = [&](int n) { return (int)std::lround((double)g->sigma * n); };
    c->mz = g->ndim == 3 ? m(c->nz) : 1;
    c->my = m(c->ny);
    c->mx = m(c->nx);
    c->N = g->nsamp;
    const double W = 4.0, s = g->sigma;
    c->beta = g->beta > 0 ? g->beta
                          : (float)(M_PI * std::sqrt((W / s) * (W / s) * (s - 0.5) * (s - 0.5) - 0.8));
  } else {
    c->mz = c->nz; c->my = c->ny; c->mx = c->nx;
    c->N = c->D;
  }
  c->M = (long long)c->mz * c->my * c->mx;
  return CS_OK;
}

// The context's work buffers: (field, bytes) in a fixed order.  They come
// from the caller's workspace (each at a 256-byte boundary) or from hipMalloc.
constexpr size_t kWsAlign = 256;
size_t ws_round(size_t b) { return (std::max<size_t>(b, 16) + kWsAlign - 1) / kWsAlign * kWsAlign; }

std::vector<std::pair<void**, size_t>> ws_requests(cs_ctx* c) {
  const size_t f2 = sizeof(float2);
  const size_t C = (size_t)c->C;
  std::vector<std::pair<void**, size_t>> r = {
      {(void**)&c->gridA, f2 * c->M * kCoilChunk},
      {(void**)&c->gridB, f2 * c->M * kCoilChunk},
      {(void**)&c->red, sizeof(double) * 2 * 1024},
      {(void**)&c->red_out, sizeof(double) * 2 * 1024},
      {(void**)&c->cov_part, sizeof(double) * 2 * 512 * C * C},
      {(void**)&c->cov, sizeof(double) * 2 * C * C},
      {(void**)&c->eig_dev, sizeof(double) * (2 * C * C + C)},
      {(void**)&c->vmaps, f2 * c->D * C},
      {(void**)&c->smaps, f2 * c->D * C},
      {(void**)&c->wav1, f2 * c->D},
      {(void**)&c->wav2, f2 * c->D},
      {(void**)&c->tvu, f2 * c->D * c->ndim}};
  c->img.assign(12, nullptr);
  for (auto& p : c->img) r.push_back({(void**)&p, f2 * c->D});
  return r;
}

int create_impl(const cs_geom* g, void* workspace, size_t ws_bytes, void* stream,
                cs_ctx** out) {
  if (!g || !out) return fail(nullptr, CS_EINVAL, "null argument");
  *out = nullptr;
  cs_ctx* c = new cs_ctx();
  int rc = init_geometry(c, g);
  if (rc != CS_OK) {
    delete c;
    return rc;
  }
  c->stream = (hipStream_t)stream;
  if (const char* e = std::getenv("CS_FFT_PIX")) c->fft_pix = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("CS_FFT_COLS")) c->fft_cols = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("CS_FFT_VEC")) c->fft_vec = std::atoi(e) != 0;
  if (const char* e = std::getenv("CS_FFT_PRO_COLS")) c->fft_pro_cols = std::atoi(e);
  if (const char* e = std::getenv("CS_FFT_VEC_IMG")) c->fft_vec_img = std::atoi(e) != 0;
  if (const char* e = std::getenv("CS_FFT_SUM_ROWS")) c->fft_sum_rows = std::atoi(e) != 0;
  if (const char* e = std::getenv("CS_GRID_VEC")) c->grid_vec = std::atoi(e) != 0;
  if (const char* e = std::getenv("CS_FFT_XCD")) c->fft_xcd = std::atoi(e) != 0;
  auto reqs = ws_requests(c);
  if (workspace) {
    size_t need = 0;
    for (auto& q : reqs) need += ws_round(q.second);
    if ((reinterpret_cast<uintptr_t>(workspace) % kWsAlign) != 0 || ws_bytes < need) {
      delete c;
      return fail(nullptr, CS_EINVAL,
                  "workspace must be 256-byte aligned and at least cs_workspace_size() bytes");
    }
    c->ws_external = true;
    char* base = static_cast<char*>(workspace);
    size_t off = 0;
    for (auto& q : reqs) {
      *q.first = base + off;
      off += ws_round(q.second);
    }
  } else {
    for (auto& q : reqs) {
      hipError_t e = hipMalloc(q.first, std::max<size_t>(q.second, 16));
      if (e != hipSuccess) {
        cs_destroy(c);
        g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
        return CS_EHIP;
      }
    }
  }
  if (hipHostMalloc((void**)&c->host_red, sizeof(double) * 2 * 1024) != hipSuccess) {
    cs_destroy(c);
    g_create_error = "hipHostMalloc failed";
    return CS_EHIP;
  }
  // scale tables: the first pass axis carries 1/sqrt(D); the non-Cartesian
  // operator divides by the KB transform Phi(r / m) per axis
  const double isd = 1.0 / std::sqrt((double)c->D);
  const int n3[3] = {c->nz, c->ny, c->nx};
  const int m3[3] = {c->mz, c->my, c->mx};
  std::vector<float> tab[3];
  for (int a = 0; a < 3; ++a) {
    tab[a].resize(n3[a]);
    for (int t = 0; t < n3[a]; ++t) {
      double v = 1.0;
      if (g->kind == CS_NONCART && !(a == 0 && c->ndim == 2))
        v = 1.0 / kb_ft((double)(t - n3[a] / 2) / (double)m3[a], 4.0, c->beta);
      tab[a][t] = (float)v;
    }
  }
  const int first = c->ndim == 3 ? 0 : 1;
  for (auto& v : tab[first]) v = (float)((double)v * isd);
  // per-pixel tables of the axes after the first
  std::vector<float> dpz((size_t)c->ny * c->nx), dpy(c->nx), y1d(c->ny);
  for (int y = 0; y < c->ny; ++y) y1d[y] = (float)(1.0 / std::sqrt((double)c->ny));
  for (int y = 0; y < c->ny; ++y)
    for (int x = 0; x < c->nx; ++x) dpz[(size_t)y * c->nx + x] = tab[1][y] * tab[2][x];
  for (int x = 0; x < c->nx; ++x) dpy[x] = tab[2][x];
  if ((rc = upload_table(c, &c->da[0], tab[0])) || (rc = upload_table(c, &c->da[1], tab[1])) ||
      (rc = upload_table(c, &c->da[2], tab[2])) || (rc = upload_table(c, &c->dp_z, dpz)) ||
      (rc = upload_table(c, &c->dp_y, dpy)) || (rc = upload_table(c, &c->da_y1d, y1d)) ||
      (rc = wavelet_init(c)) || (rc = mix_scratch_init(c)) || (rc = create_plans(c)) ||
      (rc = coil_mix_reserve(c))) {
    std::string e = c->err;
    cs_destroy(c);
    g_create_error = e;
    return rc;
  }
  *out = c;
  return CS_OK;
}

}  // namespace

int adjoint_all(cs_ctx* c, const float2* maps, int ncoil, const float2* y, float2* x) {
  return chunk_loop(c, ncoil, op_adjoint, maps, y, x);
}

int power_iter(cs_ctx* c, const float2* maps, int ncoil, int n_iter, double* L) {
  float2* v = c->img[8];
  float2* w = c->img[9];
  CS_TRY(vec_fill(c, v, c->D, (float)(1.0 / std::sqrt((double)c->D)), 0.f));
  for (int i = 0; i < n_iter; ++i) {
    CS_TRY(op_normal(c, maps, ncoil, v, w));
    double d[2];
    CS_TRY(vec_dot(c, w, w, c->D, d));
    const double nrm = std::sqrt(d[0]);
    if (!(nrm > 0) || !std::isfinite(nrm)) return fail(c, CS_ENUMERIC, "power iteration norm");
    CS_TRY(vec_axpby(c, v, (float)(1.0 / nrm), w, 0.f, w, c->D));
  }
  CS_TRY(op_normal(c, maps, ncoil, v, w));
  double d[2];
  CS_TRY(vec_dot(c, w, w, c->D, d));
  *L = std::sqrt(d[0]);
  return CS_OK;
}

// a recon buffer of at least `need` complex elements (allocates only when it
// grows: after cs_reserve_recon with enough room, never)
int grow_buf(cs_ctx* c, float2** buf, size_t* have, size_t need) {
  if (need <= *have) return CS_OK;
  if (*buf) CS_HIP(c, hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  CS_HIP(c, hipMalloc(buf, sizeof(float2) * need));
  *have = need;
  return CS_OK;
}

// virtual maps c'[d][j] = sum_c conj(U[c][j]) c[d][c] from the basis in c->U
int form_vmaps(cs_ctx* c) {
  const int C = c->C;
  std::vector<double> M((size_t)2 * C * C);
  for (int j = 0; j < C; ++j)
    for (int cc = 0; cc < C; ++cc) {
      M[2 * (j * C + cc)] = c->U[2 * (cc * C + j)];
      M[2 * (j * C + cc) + 1] = -c->U[2 * (cc * C + j) + 1];
    }
  CS_TRY(coil_mix(c, c->maps, C, 0, C, M.data(), C, c->vmaps, C, 0, 1.0f));
  c->have_U = true;
  ++c->vmaps_gen;
  return CS_OK;
}

int sketch_impl(cs_ctx* c, const float2* y, int V, int S, uint64_t seed, int t, int refresh,
                float2* smaps, std::vector<int8_t>* signs_out) {
  const int C = c->C;
  // within a compressed reconstruction the sketch acts on the first c0_active
  // virtual coils only
  const int Ce = c->c0_active > 0 ? c->c0_active : C;
  if (V < 0 || S < 0 || V + S < 1 || V + S > Ce)
    return fail(c, CS_EINVAL, "sketch sizes: need V >= 0, S >= 0 and 0 < V + S <= C");
  if (!c->have_U || refresh) {
    if (!y) return fail(c, CS_EINVAL, "y is required for the first sketch");
    CS_TRY(covariance_eig(c, y));
    CS_TRY(form_vmaps(c));
  }
  const int Ch = V + S;
  // the V identity rows (the high-energy virtual coils) are the same at
  // every outer iteration: the context's own sketched maps keep them from
  // the first draw on the current virtual maps with this layout
  const bool own = smaps == c->smaps;
  if (V > 0 && !(own && c->vrows_gen == c->vmaps_gen && c->vrows_V == V && c->vrows_Ch == Ch)) {
    std::vector<double> I((size_t)2 * V * V, 0.0);
    for (int j = 0; j < V; ++j) I[2 * (j * V + j)] = 1.0;
    CS_TRY(coil_mix(c, c->vmaps, C, 0, V, I.data(), V, smaps, Ch, 0, 1.0f));
    if (own) {
      c->vrows_gen = c->vmaps_gen;
      c->vrows_V = V;
      c->vrows_Ch = Ch;
    }
  }
  std::vector<int8_t> sg;
  if (S > 0 && V < Ce) {
    const int cols = Ce - V;
    std::vector<double> R((size_t)2 * S * cols, 0.0);
    float scale = (float)(1.0 / std::sqrt((double)S));
    if (c->inj_S == S && c->inj_V == V && c->inj_R.size() == (size_t)S * cols) {
      // injected block, used as given (its scale included)
      for (size_t e = 0; e < c->inj_R.size(); ++e) R[2 * e] = c->inj_R[e];
      scale = 1.0f;
    } else if (c->sketch_dist == CS_SKETCH_GAUSSIAN) {
      std::vector<double> gv;
      gaussian(seed, t, S, cols, gv);
      for (int a = 0; a < S; ++a)
        for (int b = 0; b < cols; ++b) R[2 * (a * cols + b)] = gv[(size_t)a * cols + b];
    } else {
      rademacher(seed, t, S, cols, sg);
      for (int a = 0; a < S; ++a)
        for (int b = 0; b < cols; ++b) R[2 * (a * cols + b)] = (double)sg[(size_t)a * cols + b];
    }
    CS_TRY(coil_mix(c, c->vmaps, C, V, cols, R.data(), S, smaps, Ch, V, scale));
  }
  if (signs_out) *signs_out = sg;
  return CS_OK;
}

int op_normal(cs_ctx* c, const float2* maps, int ncoil, const float2* x, float2* out) {
  for (int c0 = 0; c0 < ncoil; c0 += kCoilChunk) {
    const int cb = std::min(kCoilChunk, ncoil - c0);
    CS_TRY(op_normal_chunk(c, maps, ncoil, c0, cb, x, out));
  }
  return CS_OK;
}

// K FISTA iterations on the sketched subproblem of Algorithm 1,
//   min_x 1/2 ||A_S (x - x^t)||^2 + <x, d> + lambda ||Psi x||_1,
// started at x^t = x with the momentum restarted: gradient A_S^H A_S (z - x^t)
// + d, step a, prox threshold tau_l = a lambda.  d is c->img[1]; c->smaps
// holds the Ch sketched maps.  Only kernels on the context stream, no host
// synchronisation (the sequence can be captured in a graph).  `timed`, when
// given, wraps the sketched apply (kind 1) and the prox (kind 2); `start`,
// when given, is the first iterate instead of x^t.
int inner_fista(cs_ctx* c, float2* x, int Ch, int K, float a, float tau_l,
                const std::function<int(int, const std::function<int()>&)>* timed,
                const float2* start) {
  const long long D = c->D;
  float2* d = c->img[1];
  float2* z = c->img[2];
  float2* xt = c->img[3];
  float2* e = c->img[4];
  float2* g = c->img[5];
  float2* v = c->img[6];
  float2* xn = c->img[7];
  auto run = [&](int kind, const std::function<int()>& fn) {
    return timed ? (*timed)(kind, fn) : fn();
  };
  CS_TRY(vec_copy(c, xt, x, D));
  if (start) CS_TRY(vec_copy(c, x, start, D));  // warm start; the subproblem stays at x^t
  CS_TRY(vec_copy(c, z, x, D));
  double tau = 1.0;
  for (int k = 0; k < K; ++k) {
    CS_TRY(vec_axpby(c, e, 1.f, z, -1.f, xt, D));
    CS_TRY(run(1, [&] { return op_normal(c, c->smaps, Ch, e, g); }));
    CS_TRY(vec_fista_step(c, v, z, a, g, 1.f, d, D));
    CS_TRY(run(2, [&] { return prox_l1(c, v, tau_l, xn); }));
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * tau * tau)) / 2.0;
    const float beta = (float)((tau - 1.0) / tn);
    tau = tn;
    CS_TRY(vec_momentum(c, z, x, xn, beta, D));
  }
  return CS_OK;
}

// K conjugate-gradient iterations on (A^H A + lam I) u = rhs, A^H A built
// on `maps` (ncoil coils).  On entry u holds the start and r the right-hand
// side; the residual r = rhs - M u is formed here (one extra apply unless
// u_zero says u = 0).  CG scalars are FP64 reductions; p and q are work
// vectors.  Returns the normal applies made in *napplies.
int cg_solve(cs_ctx* c, const float2* maps, int ncoil, float lam, float2* u, bool u_zero,
             float2* r, float2* p, float2* q, int K, int kind,
             const std::function<int(int, const std::function<int()>&)>* timed,
             long long* napplies) {
  const long long D = c->D;
  auto run = [&](const std::function<int()>& fn) { return timed ? (*timed)(kind, fn) : fn(); };
  long long n = 0;
  if (!u_zero) {
    CS_TRY(run([&] { return op_normal(c, maps, ncoil, u, q); }));
    ++n;
    CS_TRY(vec_axpby(c, q, 1.f, q, lam, u, D));  // q = M u
    CS_TRY(vec_axpby(c, r, 1.f, r, -1.f, q, D));
  }
  CS_TRY(vec_copy(c, p, r, D));
  double rr[2];
  CS_TRY(vec_dot(c, r, r, D, rr));
  for (int k = 0; k < K; ++k) {
    if (!(rr[0] > 0.0)) break;  // exact solution (or zero right-hand side)
    CS_TRY(run([&] { return op_normal(c, maps, ncoil, p, q); }));
    ++n;
    CS_TRY(vec_axpby(c, q, 1.f, q, lam, p, D));
    double pq[2];
    CS_TRY(vec_dot(c, p, q, D, pq));
    if (!(pq[0] > 0.0) || !std::isfinite(pq[0])) break;
    const double alpha = rr[0] / pq[0];
    CS_TRY(vec_axpby(c, u, 1.f, u, (float)alpha, p, D));
    CS_TRY(vec_axpby(c, r, 1.f, r, (float)-alpha, q, D));
    double rn[2];
    CS_TRY(vec_dot(c, r, r, D, rn));
    const double beta = rn[0] / rr[0];
    CS_TRY(vec_axpby(c, p, 1.f, r, (float)beta, p, D));
    rr[0] = rn[0];
  }
  *napplies = n;
  return CS_OK;
}

}  // namespace cs

using namespace cs;

extern "C" {

int cs_create(const cs_geom* g, void* stream, cs_ctx** out) {
  return create_impl(g, nullptr, 0, stream, out);
}

int cs_workspace_size(const cs_geom* g, size_t* bytes) {
  if (!g || !bytes) return fail(nullptr, CS_EINVAL, "null argument");
  cs_ctx tmp;
  CS_TRY(init_geometry(&tmp, g));
  size_t need = 0;
  for (auto& q : ws_requests(&tmp)) need += ws_round(q.second);
  *bytes = need;
  return CS_OK;
}

int cs_create_ws(const cs_geom* g, void* workspace, size_t ws_bytes, void* stream,
                 cs_ctx** out) {
  if (!workspace) return fail(nullptr, CS_EINVAL, "workspace is null");
  return create_impl(g, workspace, ws_bytes, stream, out);
}

void cs_destroy(cs_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  if (!c->ws_external) {  // buffers carved from a caller's workspace stay theirs
    fr(c->gridA); fr(c->gridB); fr(c->red); fr(c->red_out);
    fr(c->cov_part); fr(c->cov); fr(c->eig_dev); fr(c->vmaps); fr(c->smaps);
    fr(c->wav1); fr(c->wav2); fr(c->tvu);
    for (auto* p : c->img) fr(p);
  }
  fr(c->mask); fr(c->rec); fr(c->vbuf); fr(c->dcf_orig);
  fr(c->mixB); fr(c->ones);
  for (int k = 0; k < cs_ctx::kStage; ++k) {
    if (c->stage[k]) (void)hipHostFree(c->stage[k]);
    if (c->stage_ev[k]) (void)hipEventDestroy(c->stage_ev[k]);
  }
  fr(c->gitems); fr(c->item_off); fr(c->partial);
  for (int a = 0; a < 3; ++a) fr(c->da[a]);
  fr(c->dp_z); fr(c->dp_y); fr(c->da_y1d);
  fr(c->ysk);
  fr(c->cmaps);
  fr(c->ycmp);
  for (auto& kv : c->plans) fr(kv.second.tw);
  if (c->host_red) (void)hipHostFree(c->host_red);
  for (auto& r : c->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

const char* cs_last_error(const cs_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

int cs_set_operator(cs_ctx* c, const void* maps, const uint8_t* mask, const float* coords,
                    const float* dcf) {
  if (!c) return CS_EINVAL;
  if (!maps) return fail(c, CS_EINVAL, "maps is null");
  CS_HIP(c, hipStreamSynchronize(c->stream));
  // the context has no operator until this call succeeds
  c->have_op = false;
  c->maps = (const float2*)maps;
  c->have_U = false;
  c->have_b = false;
  if (c->g.kind == CS_CART) {
    if (!mask) return fail(c, CS_EINVAL, "Cartesian operator needs a mask");
    std::vector<uint8_t> h(c->D);
    CS_HIP(c, hipMemcpy(h.data(), mask, c->D, hipMemcpyDeviceToHost));
    bool oned = true;
    for (int y = 0; y < c->ny && oned; ++y)
      for (int x = 1; x < c->nx; ++x)
        if ((h[(size_t)y * c->nx + x] != 0) != (h[(size_t)y * c->nx] != 0)) {
          oned = false;
          break;
        }
    for (auto& v : h) v = v ? 1 : 0;
    if (!c->mask) CS_HIP(c, hipMalloc(&c->mask, c->D));
    CS_HIP(c, hipMemcpy(c->mask, h.data(), c->D, hipMemcpyHostToDevice));
    c->mask1d = oned;
  } else {
    if (!coords && c->N > 0) return fail(c, CS_EINVAL, "non-Cartesian operator needs coordinates");
    if (c->rec) {
      CS_HIP(c, hipFree(c->rec)); c->rec = nullptr;
      CS_HIP(c, hipFree(c->vbuf)); c->vbuf = nullptr;
      CS_HIP(c, hipFree(c->gitems)); c->gitems = nullptr;
      CS_HIP(c, hipFree(c->item_off)); c->item_off = nullptr;
      CS_HIP(c, hipFree(c->partial)); c->partial = nullptr;
      c->n_items = 0;
      c->partial_elems = 0;
      c->group_off.clear();
    }
    if (c->dcf_orig) {
      CS_HIP(c, hipFree(c->dcf_orig));
      c->dcf_orig = nullptr;
    }
    CS_TRY(setup_noncart(c, coords, dcf));
  }
  c->have_op = true;
  return CS_OK;
}

int sense_apply(cs_ctx* c, const void* maps, int ncoil, const void* x, void* y) {
  CS_TRY(check_ready(c, maps, ncoil, x, y, 2));
  return chunk_loop(c, ncoil, op_apply, (const float2*)maps, (const float2*)x, (float2*)y);
}

int sense_adjoint(cs_ctx* c, const void* maps, int ncoil, const void* y, void* x) {
  CS_TRY(check_ready(c, maps, ncoil, y, x, 1));
  return chunk_loop(c, ncoil, op_adjoint, (const float2*)maps, (const float2*)y, (float2*)x);
}

int normal_apply(cs_ctx* c, const void* maps, int ncoil, const void* x, void* out) {
  CS_TRY(check_ready(c, maps, ncoil, x, out));
  if (x == out) return fail(c, CS_EINVAL, "x and out must not alias");
  return op_normal(c, (const float2*)maps, ncoil, (const float2*)x, (float2*)out);
}

int sketch_build(cs_ctx* c, const void* y, int V, int S, uint64_t seed, int t, int refresh,
                 void* smaps, double* eig, double* U_out, int8_t* signs) {
  if (!c) return CS_EINVAL;
  if (!c->have_op) return fail(c, CS_EINVAL, "cs_set_operator has not been called");
  if (!smaps) return fail(c, CS_EINVAL, "smaps is null");
  std::vector<int8_t> sg;
  CS_TRY(sketch_impl(c, (const float2*)y, V, S, seed, t, refresh, (float2*)smaps, &sg));
  if (eig) std::memcpy(eig, c->lam.data(), sizeof(double) * c->C);
  if (U_out) std::memcpy(U_out, c->U.data(), sizeof(double) * 2 * c->C * c->C);
  if (signs && !sg.empty()) std::memcpy(signs, sg.data(), sg.size());
  if (eig || U_out || signs) CS_HIP(c, hipStreamSynchronize(c->stream));
  return CS_OK;
}

int cs_reserve_recon(cs_ctx* c, int C0, int init_coils) {
  if (!c) return CS_EINVAL;
  if (C0 < 0 || C0 > c->C || init_coils < 0 || init_coils > c->C)
    return fail(c, CS_EINVAL, "cs_reserve_recon: C0 and init_coils must be in [0, C]");
  const size_t Nd = (size_t)std::max(1LL, c->N);
  if (C0 > 0) {
    CS_TRY(grow_buf(c, &c->cmaps, &c->cmaps_elems, (size_t)c->D * C0));
    CS_TRY(grow_buf(c, &c->ycmp, &c->ycmp_elems, Nd * C0));
  }
  if (init_coils > 0) CS_TRY(grow_buf(c, &c->ysk, &c->ysk_elems, Nd * init_coils));
  return CS_OK;
}

int cs_set_basis(cs_ctx* c, const double* U, const double* lam) {
  if (!c) return CS_EINVAL;
  if (!c->have_op) return fail(c, CS_EINVAL, "cs_set_operator has not been called");
  if (!U) return fail(c, CS_EINVAL, "U is null");
  const int C = c->C;
  for (int i = 0; i < 2 * C * C; ++i)
    if (!std::isfinite(U[i])) return fail(c, CS_EINVAL, "U has a non-finite entry");
  c->U.assign(U, U + 2 * C * C);
  if (lam) c->lam.assign(lam, lam + C);
  else c->lam.assign(C, 0.0);
  return form_vmaps(c);
}

int cs_set_sketch(cs_ctx* c, int V, int S, const double* R) {
  if (!c) return CS_EINVAL;
  if (!R) {
    c->inj_R.clear();
    c->inj_V = c->inj_S = -1;
    return CS_OK;
  }
  if (V < 0 || S < 1 || V + S > c->C || V >= c->C)
    return fail(c, CS_EINVAL, "cs_set_sketch: need V >= 0, S >= 1, V + S <= C and V < C");
  const size_t n = (size_t)S * (c->C - V);
  for (size_t e = 0; e < n; ++e)
    if (!std::isfinite(R[e])) return fail(c, CS_EINVAL, "R has a non-finite entry");
  c->inj_R.assign(R, R + n);
  c->inj_V = V;
  c->inj_S = S;
  return CS_OK;
}

int cs_set_sketch_dist(cs_ctx* c, int dist) {
  if (!c) return CS_EINVAL;
  if (dist != CS_SKETCH_RADEMACHER && dist != CS_SKETCH_GAUSSIAN)
    return fail(c, CS_EINVAL, "sketch distribution");
  c->sketch_dist = dist;
  return CS_OK;
}

int cs_prox_l1wav(cs_ctx* c, const void* v, float tau, void* out) {
  if (!c || !v || !out) return CS_EINVAL;
  return prox_l1(c, (const float2*)v, tau, (float2*)out);
}

int cs_dwt(cs_ctx* c, const void* x, void* coef) {
  if (!c || !x || !coef) return CS_EINVAL;
  return dwt_fwd(c, (const float2*)x, (float2*)coef);
}

int cs_idwt(cs_ctx* c, const void* coef, void* x) {
  if (!c || !x || !coef) return CS_EINVAL;
  return dwt_inv(c, (const float2*)coef, (float2*)x);
}

int cs_coil_mix(cs_ctx* c, const void* in, int cin, const double* M, int cout, void* out) {
  if (!c || !in || !M || !out) return CS_EINVAL;
  return coil_mix(c, (const float2*)in, cin, 0, cin, M, cout, (float2*)out, cout, 0, 1.0f);
}

int cs_coil_mix_noalloc(cs_ctx* c, const void* in, int cin, const void* M, int cout,
                        void* out) {
  if (!c) return CS_EINVAL;
  if (!in || !M || !out) return fail(c, CS_EINVAL, "null pointer");
  return coil_mix_noalloc(c, (const float2*)in, cin, M, cout, (float2*)out);
}

int cs_dot(cs_ctx* c, const void* a, const void* b, double* out) {
  if (!c || !a || !b || !out) return CS_EINVAL;
  return vec_dot(c, (const float2*)a, (const float2*)b, c->D, out);
}

int cs_power_iteration(cs_ctx* c, const void* maps, int ncoil, int n_iter, double* L) {
  CS_TRY(check_ready(c, maps, ncoil, maps, maps));
  if (!L || n_iter < 0) return fail(c, CS_EINVAL, "power iteration arguments");
  return power_iter(c, (const float2*)maps, ncoil, n_iter, L);
}

int cs_grid_shape(const cs_ctx* c, int m[3]) {
  if (!c || !m) return CS_EINVAL;
  m[0] = c->mz; m[1] = c->my; m[2] = c->mx;
  return CS_OK;
}

int cs_profile_enable(cs_ctx* c, int on) {
  if (!c) return CS_EINVAL;
  c->prof = on != 0;
  return CS_OK;
}

int cs_profile_read(cs_ctx* c, double* ms, long long* count) {
  if (!c) return CS_EINVAL;
  CS_HIP(c, hipStreamSynchronize(c->stream));
  for (auto& r : c->prof_recs) {
    float t = 0.f;
    CS_HIP(c, hipEventElapsedTime(&t, r.a, r.b));
    c->prof_ms[r.kind] += t;
    c->prof_cnt[r.kind] += 1;
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof_recs.clear();
  for (int k = 0; k < CS_NKERNELS; ++k) {
    if (ms) ms[k] = c->prof_ms[k];
    if (count) count[k] = c->prof_cnt[k];
    c->prof_ms[k] = 0.0;
    c->prof_cnt[k] = 0;
  }
  return CS_OK;
}

}  // extern "C"

namespace cs {
// Scales of the network's inputs and output: s_d = rms(d); s_o = alpha rms(d),
// the size of one gradient step, which is the unit of the predicted change;
// s_x = rms(x), or s_o while x = 0.  A vanishing scale is replaced by 1.
int warm_scales(cs_ctx* c, const float2* x, const float2* d, double alpha, double* sx,
                double* sd, double* so) {
  double xx[2], dd[2];
  CS_TRY(vec_dot(c, x, x, c->D, xx));
  CS_TRY(vec_dot(c, d, d, c->D, dd));
  const double rx = std::sqrt(xx[0] / (double)c->D), rd = std::sqrt(dd[0] / (double)c->D);
  *sd = rd > 0 ? rd : 1.0;
  *so = alpha * rd > 0 ? alpha * rd : 1.0;
  *sx = rx > 0 ? rx : *so;
  return CS_OK;
}
}  // namespace cs

extern "C" {

int cs_cnn_collect(cs_ctx* c, const void* y_, const cs_recon_params* p, void* x_inout,
                   float* inputs, float* targets) {
  if (!c) return CS_EINVAL;
  if (!c->have_op) return fail(c, CS_EINVAL, "cs_set_operator has not been called");
  if (!y_ || !p || !x_inout || !inputs || !targets) return fail(c, CS_EINVAL, "null argument");
  if (p->T < 1 || p->K < 1) return fail(c, CS_EINVAL, "iteration counts");
  if (p->reg != CS_REG_L1WAV) return fail(c, CS_EINVAL, "pairs are collected for l1-wavelet only");
  if ((p->C0 > 0 && p->C0 < c->C) || p->init_iters != 0 || p->monitor != 0)
    return fail(c, CS_EINVAL,
                "pairs are collected on all coils, without compression, the "
                "classical-sketch initialisation or the objective monitor");
  const float2* y = (const float2*)y_;
  float2* x = (float2*)x_inout;
  const long long D = c->D;
  float2* b = c->img[0];
  float2* d = c->img[1];
  float2* g = c->img[5];
  float2* xo = c->img[8];
  const int Ch = p->V + p->S;
  CS_TRY(adjoint_all(c, c->maps, c->C, y, b));
  c->have_b = true;
  c->b_c0 = c->C;  // b is over every coil: a compressed recon_run must not reuse it
  CS_TRY(sketch_impl(c, y, p->V, p->S, p->seed, p->t0, 0, c->smaps, nullptr));
  double alpha = p->step;
  if (alpha <= 0) {
    double L = 0;
    CS_TRY(power_iter(c, c->smaps, Ch, p->n_pow > 0 ? p->n_pow : 30, &L));
    alpha = 1.0 / L;
  }
  for (int it = 0; it < p->T; ++it) {
    CS_TRY(op_normal(c, c->maps, c->C, x, g));
    CS_TRY(vec_axpby(c, d, 1.f, g, -1.f, b, D));
    if (it > 0) CS_TRY(sketch_impl(c, y, p->V, p->S, p->seed, p->t0 + it, 0, c->smaps, nullptr));
    double sx, sd, so;
    CS_TRY(warm_scales(c, x, d, alpha, &sx, &sd, &so));
    CS_TRY(cnn_pack_input(c, x, d, (float)sx, (float)sd, inputs + (size_t)it * D * 4));
    CS_TRY(vec_copy(c, xo, x, D));
    CS_TRY(inner_fista(c, x, Ch, p->K, (float)alpha, (float)(alpha * p->lam), nullptr, nullptr));
    CS_TRY(cnn_pack_target(c, x, xo, (float)so, targets + (size_t)it * D * 2));
  }
  CS_HIP(c, hipStreamSynchronize(c->stream));
  return CS_OK;
}

int recon_run(cs_ctx* c, const void* y_, const cs_recon_params* p, void* x_inout,
              cs_recon_stats* st) {
  if (!c) return CS_EINVAL;
  if (!c->have_op) return fail(c, CS_EINVAL, "cs_set_operator has not been called");
  if (!y_ || !p || !x_inout) return fail(c, CS_EINVAL, "null argument");
  if (p->mode != CS_RECON_FULL && p->mode != CS_RECON_SKETCH &&
      p->mode != CS_RECON_SKETCH_LEARNED)
    return fail(c, CS_EINVAL, "recon mode");
  const bool learned = p->mode == CS_RECON_SKETCH_LEARNED;
  if (learned && !p->cnn) return fail(c, CS_EINVAL, "learned mode needs a network");
  if (p->reg != CS_REG_L1WAV && p->reg != CS_REG_L2 && p->reg != CS_REG_TV)
    return fail(c, CS_EINVAL, "regularizer");
  const bool l2 = p->reg == CS_REG_L2;
  const bool tvr = p->reg == CS_REG_TV;
  if ((l2 || tvr) && learned)
    return fail(c, CS_EINVAL, "the learned warm start is for l1-wavelet only");
  if (p->init_iters < 0 ||
      (p->init_iters > 0 && (l2 || tvr || p->mode == CS_RECON_FULL)))
    return fail(c, CS_EINVAL, "the classical-sketch initialisation is for l1-wavelet Algorithm 1");
  if (p->monitor && (l2 || tvr || p->mode == CS_RECON_FULL))
    return fail(c, CS_EINVAL, "the objective monitor is for l1-wavelet Algorithm 1");
  if (p->monitor && !(p->mon_tol >= 0.0)) return fail(c, CS_EINVAL, "mon_tol must be >= 0");
  if (p->C0 < 0) return fail(c, CS_EINVAL, "C0");
  if (p->C0 > 0 && p->C0 < c->C && p->init_iters > 0)
    return fail(c, CS_EINVAL, "the classical-sketch initialisation needs C0 = C");
  if (p->C0 > 0 && p->C0 < c->C && p->mode != CS_RECON_FULL && p->V + p->S > p->C0)
    return fail(c, CS_EINVAL, "sketch sizes: need V + S <= C0");
  if (p->T < 0 || (p->mode != CS_RECON_FULL && p->K < 1))
    return fail(c, CS_EINVAL, "iteration counts");
  if (st) {
    st->n_warm_accepted = st->n_warm_rejected = 0;
    st->n_fallbacks = 0;
    st->objective0 = 0.0;
    st->ms_monitor = 0.0;
  }
  const float2* y = (const float2*)y_;
  float2* x = (float2*)x_inout;
  const long long D = c->D;
  const int C = c->C;
  float2* b = c->img[0];
  float2* d = c->img[1];
  float2* z = c->img[2];
  float2* g = c->img[5];
  float2* v = c->img[6];
  float2* xn = c->img[7];
  // pooled events taken by this call go back to the pool on every return path
  struct PoolBack {
    cs_ctx* c;
    std::vector<hipEvent_t> evs;
    ~PoolBack() {
      for (auto q : evs) c->ev_pool.push_back(q);
    }
  } pooled{c, {}};
  hipEvent_t ev_prep = pool_event(c);
  if (!ev_prep) return fail(c, CS_EHIP, "event creation failed");
  pooled.evs.push_back(ev_prep);
  CS_HIP(c, hipEventRecord(ev_prep, c->stream));
  // Alg. 1's initial coil compression: the model and the data rotated onto
  // the first C0 PCA virtual coils; the full-coil operator below is then
  // (fmaps, FC) and the sketches draw over those FC virtual coils
  const bool compress = p->C0 > 0 && p->C0 < C;
  struct C0Scope {
    cs_ctx* c;
    ~C0Scope() { c->c0_active = 0; }
  } c0scope{c};
  const float2* fmaps = c->maps;
  int FC = C;
  if (compress) {
    const int C0 = p->C0;
    if (!c->have_U) CS_TRY(sketch_impl(c, y, C0, 0, p->seed, p->t0, 0, c->smaps, nullptr));
    CS_TRY(grow_buf(c, &c->cmaps, &c->cmaps_elems, (size_t)c->D * C0));
    CS_TRY(grow_buf(c, &c->ycmp, &c->ycmp_elems, (size_t)std::max(1LL, c->N) * C0));
    // first C0 rows of U^H: M[j][cc] = conj(U[cc][j])
    std::vector<double> M((size_t)2 * C0 * C);
    for (int j = 0; j < C0; ++j)
      for (int cc = 0; cc < C; ++cc) {
        M[2 * (j * C + cc)] = c->U[2 * (cc * C + j)];
        M[2 * (j * C + cc) + 1] = -c->U[2 * (cc * C + j) + 1];
      }
    std::vector<double> I((size_t)2 * C0 * C0, 0.0);
    for (int j = 0; j < C0; ++j) I[2 * (j * C0 + j)] = 1.0;
    CS_TRY(coil_mix(c, c->vmaps, C, 0, C0, I.data(), C0, c->cmaps, C0, 0, 1.0f));
    CS_TRY(coil_mix_rows(c, c->N, y, C, 0, C, M.data(), C0, c->ycmp, C0, 0, 1.0f));
    c->c0_active = C0;
    fmaps = c->cmaps;
    FC = C0;
  }
  if (!p->reuse_b || !c->have_b || c->b_c0 != FC) {
    if (compress)
      CS_TRY(chunk_loop(c, FC, op_adjoint, fmaps, c->ycmp, b));
    else
      CS_TRY(chunk_loop(c, C, op_adjoint, c->maps, y, b));
    c->have_b = true;
    c->b_c0 = FC;
  }
  const int Ch = p->V + p->S;
  const int n_pow = p->n_pow > 0 ? p->n_pow : 30;
  long long nfull = 0, nsk = 0, nprox = 0;
  double alpha = p->step;
  if (l2 || tvr) alpha = 0.0;  // CG and PDHG need no FISTA step
  if (p->mode != CS_RECON_FULL) {
    CS_TRY(sketch_impl(c, y, p->V, p->S, p->seed, p->t0, 0, c->smaps, nullptr));
    if (alpha <= 0 && !l2 && !tvr) {
      double L = 0;
      CS_TRY(power_iter(c, c->smaps, Ch, n_pow, &L));
      nsk += n_pow + 1;
      alpha = 1.0 / L;
    }
  } else if (alpha <= 0 && !l2 && !tvr) {
    double L = 0;
    CS_TRY(power_iter(c, fmaps, FC, n_pow, &L));
    nfull += n_pow + 1;
    alpha = 1.0 / L;
  }
  const float a = (float)alpha;
  const float tau_l = (float)(alpha * p->lam);
  if (p->init_iters > 0) {
    // Alg. 1's initialisation: x^1 = argmin 1/2 ||S^0 A x - S^0 y||^2 + g(x)
    // with the structured sketch of t = 0 on the maps and on the data,
    // by plain FISTA with the first subproblem's step
    const int V = p->V, S = p->S, cols = C - p->V;
    std::vector<double> R((size_t)S * std::max(cols, 0), 0.0);
    if (S > 0) {
      if (c->sketch_dist == CS_SKETCH_GAUSSIAN) {
        gaussian(p->seed, 0, S, cols, R);
      } else {
        std::vector<int8_t> sg;
        rademacher(p->seed, 0, S, cols, sg);
        for (size_t k = 0; k < sg.size(); ++k) R[k] = sg[k];
      }
    }
    // M[j][c] = (S~^0 U^H)[j][c]: rows j < V select virtual coil j, rows
    // V + i combine the virtual coils V.. with R[i][.] / sqrt(S)
    std::vector<double> M((size_t)2 * Ch * C, 0.0);
    const double rs = S > 0 ? 1.0 / std::sqrt((double)S) : 0.0;
    for (int cc = 0; cc < C; ++cc) {
      for (int j = 0; j < V; ++j) {
        M[2 * (j * C + cc)] = c->U[2 * (cc * C + j)];
        M[2 * (j * C + cc) + 1] = -c->U[2 * (cc * C + j) + 1];
      }
      for (int i = 0; i < S; ++i)
        for (int bb = 0; bb < cols; ++bb) {
          const double w = R[(size_t)i * cols + bb] * rs;
          M[2 * ((V + i) * C + cc)] += w * c->U[2 * (cc * C + V + bb)];
          M[2 * ((V + i) * C + cc) + 1] -= w * c->U[2 * (cc * C + V + bb) + 1];
        }
    }
    CS_TRY(grow_buf(c, &c->ysk, &c->ysk_elems, (size_t)std::max(1LL, c->N) * Ch));
    CS_TRY(coil_mix_rows(c, c->N, y, C, 0, C, M.data(), Ch, c->ysk, Ch, 0, 1.0f));
    CS_TRY(sketch_impl(c, y, p->V, p->S, p->seed, 0, 0, c->smaps, nullptr));
    float2* bs = c->img[10];
    CS_TRY(chunk_loop(c, Ch, op_adjoint, c->smaps, c->ysk, bs));
    float2* z0 = c->img[2];
    float2* g0 = c->img[5];
    float2* v0 = c->img[6];
    float2* x0n = c->img[7];
    CS_TRY(vec_copy(c, z0, x, D));
    double tau = 1.0;
    for (int k = 0; k < p->init_iters; ++k) {
      CS_TRY(op_normal(c, c->smaps, Ch, z0, g0));
      ++nsk;
      CS_TRY(vec_fista_step(c, v0, z0, a, g0, -1.f, bs, D));
      CS_TRY(prox_l1(c, v0, tau_l, x0n));
      ++nprox;
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * tau * tau)) / 2.0;
      const float beta = (float)((tau - 1.0) / tn);
      tau = tn;
      CS_TRY(vec_momentum(c, z0, x, x0n, beta, D));
    }
    // the loop's first subproblem uses the sketch of t0 again
    CS_TRY(sketch_impl(c, y, p->V, p->S, p->seed, p->t0, 0, c->smaps, nullptr));
  }
  // per-call events, destroyed on every return path
  struct Events {
    std::vector<hipEvent_t> all;
    ~Events() {
      for (auto q : all) (void)hipEventDestroy(q);
    }
    hipEvent_t make() {
      hipEvent_t q = nullptr;
      if (hipEventCreate(&q) != hipSuccess) return nullptr;
      all.push_back(q);
      return q;
    }
  } owned;
  hipEvent_t ev0 = owned.make(), ev_end = owned.make();
  std::vector<hipEvent_t> ev(std::max(1, p->T)), evd(ev.size());
  for (auto& q : ev) q = owned.make();
  for (auto& q : evd) q = owned.make();
  if (owned.all.size() != 2 + 2 * ev.size()) return fail(c, CS_EHIP, "event creation failed");
  const bool track = p->x_ref != nullptr;
  std::vector<double> dist_num(p->T, 0.0), dist_den(p->T, 1.0);
  // phase timing: events around each full / sketched normal apply, prox and
  // sketch formation
  struct Phase {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Phase> phases;
  auto timed = [&](int kind, auto&& fn) -> int {
    Phase ph{kind, pool_event(c), pool_event(c)};
    if (ph.a) pooled.evs.push_back(ph.a);
    if (ph.b) pooled.evs.push_back(ph.b);
    if (!ph.a || !ph.b) return fail(c, CS_EHIP, "event creation failed");
    CS_HIP(c, hipEventRecord(ph.a, c->stream));
    const int r = fn();
    CS_HIP(c, hipEventRecord(ph.b, c->stream));
    phases.push_back(ph);
    return r;
  };
  const std::function<int(int, const std::function<int()>&)> timed_fn =
      [&](int kind, const std::function<int()>& fn) { return timed(kind, fn); };
  CS_HIP(c, hipEventRecord(ev0, c->stream));
  int rc = CS_OK;
  auto record = [&](int it) -> int {
    CS_HIP(c, hipEventRecord(ev[it], c->stream));
    if (track) {
      double num = 0, den = 0;
      CS_TRY(vec_dist(c, x, (const float2*)p->x_ref, D, &num, &den));
      dist_num[it] = num;
      dist_den[it] = den;
    }
    CS_HIP(c, hipEventRecord(evd[it], c->stream));
    return CS_OK;
  };
  if (tvr) {
    // PDHG on G + lam ||T x||_1 (theta = 1, tau = sigma = 1/sqrt(4 ndim));
    // G's prox is the CG solve of (N + I/tau) x = rhs0 + v/tau, with N and
    // rhs0 = b (plain problem) or N_S and N_S x^t - d (subproblem)
    const double step = 1.0 / std::sqrt(4.0 * c->ndim);
    const float tau = (float)step, sigma = (float)step, itau = (float)(1.0 / step);
    const int n_cg = p->n_cg > 0 ? p->n_cg : 5;
    float2* pd = c->img[2];
    float2* xbar = c->img[3];
    float2* xold = c->img[4];
    float2* q = c->img[5];
    float2* r = c->img[6];
    float2* v = c->img[7];
    float2* rhs0 = c->img[10];
    float2* xt = c->img[11];
    auto pdhg = [&](const float2* maps, int ncoil, int K, int kind, long long* napp,
                    int rec_base) -> int {
      CS_TRY(vec_fill(c, c->tvu, D * c->ndim, 0.f, 0.f));
      CS_TRY(vec_copy(c, xbar, x, D));
      for (int k = 0; k < K; ++k) {
        CS_TRY(tv_dual_step(c, c->tvu, xbar, sigma, p->lam));
        CS_TRY(tv_primal_step(c, v, x, c->tvu, tau));
        CS_TRY(vec_copy(c, xold, x, D));
        CS_TRY(vec_axpby(c, r, 1.f, rhs0, itau, v, D));
        long long n = 0;
        CS_TRY(cg_solve(c, maps, ncoil, itau, x, false, r, pd, q, n_cg, kind, &timed_fn, &n));
        *napp += n;
        CS_TRY(vec_axpby(c, xbar, 2.f, x, -1.f, xold, D));
        if (rec_base >= 0) CS_TRY(record(rec_base + k));
      }
      return CS_OK;
    };
    if (p->mode == CS_RECON_FULL) {
      CS_TRY(vec_copy(c, rhs0, b, D));
      CS_TRY(pdhg(fmaps, FC, p->T, 0, &nfull, 0));
    } else {
      for (int it = 0; it < p->T; ++it) {
        const int t = p->t0 + it;
        CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, x, g); }));
        ++nfull;
        CS_TRY(vec_axpby(c, d, 1.f, g, -1.f, b, D));
        if (it > 0)
          CS_TRY(timed(3, [&] {
            return sketch_impl(c, y, p->V, p->S, p->seed, t, 0, c->smaps, nullptr);
          }));
        CS_TRY(vec_copy(c, xt, x, D));
        CS_TRY(timed(1, [&] { return op_normal(c, c->smaps, Ch, xt, rhs0); }));
        ++nsk;
        CS_TRY(vec_axpby(c, rhs0, 1.f, rhs0, -1.f, d, D));
        long long n = 0;
        CS_TRY(pdhg(c->smaps, Ch, p->K, 1, &n, -1));
        nsk += n;
        CS_TRY(record(it));
      }
    }
  } else if (l2 && p->mode == CS_RECON_FULL) {
    // CG on (A^H A + lam I) x = b, one iteration per record
    float2* r = c->img[6];
    float2* pd = c->img[2];
    float2* q = c->img[5];
    CS_TRY(vec_copy(c, r, b, D));
    long long n = 0;
    // the first call forms the residual; later calls continue the same CG
    // (they are split only to record per-iteration progress)
    double rr[2] = {0, 0};
    for (int it = 0; it < p->T; ++it) {
      if (it == 0) {
        CS_TRY(cg_solve(c, fmaps, FC, p->lam, x, false, r, pd, q, 1, 0, &timed_fn, &n));
        nfull += n;
        CS_TRY(vec_dot(c, r, r, D, rr));
      } else if (rr[0] > 0.0) {
        CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, pd, q); }));
        ++nfull;
        CS_TRY(vec_axpby(c, q, 1.f, q, p->lam, pd, D));
        double pq[2];
        CS_TRY(vec_dot(c, pd, q, D, pq));
        if (pq[0] > 0.0 && std::isfinite(pq[0])) {
          const double al = rr[0] / pq[0];
          CS_TRY(vec_axpby(c, x, 1.f, x, (float)al, pd, D));
          CS_TRY(vec_axpby(c, r, 1.f, r, (float)-al, q, D));
          double rn[2];
          CS_TRY(vec_dot(c, r, r, D, rn));
          CS_TRY(vec_axpby(c, pd, 1.f, r, (float)(rn[0] / rr[0]), pd, D));
          rr[0] = rn[0];
        } else {
          rr[0] = 0.0;
        }
      }
      CS_TRY(record(it));
    }
  } else if (l2) {
    // Algorithm 1 with g = lam/2 ||x||^2: the subproblem of Eq. 10 is the
    // system (A_S^H A_S + lam I) u = -(d + lam x^t), K CG iterations from u = 0
    float2* u = c->img[4];
    float2* r = c->img[6];
    float2* pd = c->img[2];
    float2* q = c->img[5];
    for (int it = 0; it < p->T; ++it) {
      const int t = p->t0 + it;
      CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, x, g); }));
      ++nfull;
      CS_TRY(vec_axpby(c, d, 1.f, g, -1.f, b, D));
      if (it > 0)
        CS_TRY(timed(3, [&] {
          return sketch_impl(c, y, p->V, p->S, p->seed, t, 0, c->smaps, nullptr);
        }));
      CS_TRY(vec_axpby(c, r, -1.f, d, -p->lam, x, D));
      CS_TRY(vec_fill(c, u, D, 0.f, 0.f));
      long long n = 0;
      CS_TRY(cg_solve(c, c->smaps, Ch, p->lam, u, true, r, pd, q, p->K, 1, &timed_fn, &n));
      nsk += n;
      CS_TRY(vec_axpby(c, x, 1.f, x, 1.f, u, D));
      CS_TRY(record(it));
    }
  } else if (p->mode == CS_RECON_FULL) {
    // plain FISTA: g = A^H A z - b
    CS_TRY(vec_copy(c, z, x, D));
    double tau = 1.0;
    for (int it = 0; it < p->T && rc == CS_OK; ++it) {
      CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, z, g); }));
      ++nfull;
      CS_TRY(vec_fista_step(c, v, z, a, g, -1.f, b, D));
      CS_TRY(timed(2, [&] { return prox_l1(c, v, tau_l, xn); }));
      ++nprox;
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * tau * tau)) / 2.0;
      const float beta = (float)((tau - 1.0) / tn);
      tau = tn;
      CS_TRY(vec_momentum(c, z, x, xn, beta, D));
      CS_TRY(record(it));
    }
  } else {
    // learned warm start: z0 = x^t + s_o CNN(x^t / s_x, d^t / s_d) is used
    // as the first inner iterate only when the FP64 subproblem objective
    //   phi(u) = 1/2 <u - x^t, A_S^H A_S (u - x^t)> + Re<u, d> + lam ||Psi u||_1
    // at z0 is no larger than at x^t; otherwise the plain start is kept
    long long n_acc = 0, n_rej = 0;
    auto learned_start = [&](const float2*& warm) -> int {
      double sx, sd, so;
      CS_TRY(warm_scales(c, x, d, alpha, &sx, &sd, &so));
      float2* z0 = c->img[8];
      float2* e = c->img[9];
      float2* coef = c->img[6];
      CS_TRY(cnn_warm_start(p->cnn, c, x, d, (float)sx, (float)sd, (float)so, z0));
      CS_TRY(vec_axpby(c, e, 1.f, z0, -1.f, x, D));
      CS_TRY(op_normal(c, c->smaps, Ch, e, g));
      ++nsk;
      double q[2], lz[2], lx[2], l1z = 0, l1x = 0;
      CS_TRY(vec_dot(c, e, g, D, q));
      CS_TRY(vec_dot(c, z0, d, D, lz));
      CS_TRY(vec_dot(c, x, d, D, lx));
      CS_TRY(dwt_fwd(c, z0, coef));
      CS_TRY(vec_abs_sum(c, coef, D, &l1z));
      CS_TRY(dwt_fwd(c, x, coef));
      CS_TRY(vec_abs_sum(c, coef, D, &l1x));
      const double phz = 0.5 * q[0] + lz[0] + p->lam * l1z;
      const double phx = lx[0] + p->lam * l1x;
      if (std::isfinite(phz) && phz <= phx) {
        warm = z0;
        ++n_acc;
      } else {
        warm = nullptr;
        ++n_rej;
      }
      return CS_OK;
    };
    // objective monitor (no counterpart in the paper): with g = A^H A x from
    // the true gradient's apply,
    //   F(x) = 1/2 <x, g> - Re<x, b> + 1/2 ||y||^2 + lam ||Psi x||_1
    // (= 1/2 ||A x - y||^2 + lam ||Psi x||_1, Eqs. 3-4).  The iterate left by
    // an outer iteration is replaced, when its F is not finite or rose by
    // more than mon_tol |F(x^t)|, by the full-coil proximal-gradient step
    // x^t - d^t / L, prox_{lam / L}, whose step 1/L (L of the full operator)
    // cannot raise F
    const bool mon = p->monitor != 0;
    float2* xprev = c->img[10];
    float2* dprev = c->img[11];
    double yy = 0.0, fprev = 0.0, f0 = 0.0, af = 0.0;
    long long n_fb = 0;
    std::vector<double> fobj;
    if (mon && c->N > 0) {
      const float2* ydata = compress ? c->ycmp : y;
      double o[2];
      CS_TRY(timed(5, [&] { return vec_dot(c, ydata, ydata, c->N * FC, o); }));
      yy = o[0];
    }
    auto objective = [&](double* f) -> int {
      double xg[2], xb[2], l1 = 0.0;
      CS_TRY(vec_dot(c, x, g, D, xg));
      CS_TRY(vec_dot(c, x, b, D, xb));
      CS_TRY(dwt_fwd(c, x, v));
      CS_TRY(vec_abs_sum(c, v, D, &l1));
      *f = 0.5 * xg[0] - xb[0] + 0.5 * yy + p->lam * l1;
      return CS_OK;
    };
    // x, g and d hold the iterate left by outer iteration it and its gradient
    // pair; xprev, dprev those of the iterate it started from
    auto monitor = [&](int it) -> int {
      double f = 0.0;
      CS_TRY(timed(5, [&] { return objective(&f); }));
      if (!std::isfinite(f) || f > fprev + p->mon_tol * std::fabs(fprev)) {
        if (af <= 0.0) {
          double L = 0.0;
          CS_TRY(timed(0, [&] { return power_iter(c, fmaps, FC, n_pow, &L); }));
          nfull += n_pow + 1;
          af = 1.0 / L;
        }
        CS_TRY(timed(5, [&] {
          CS_TRY(vec_fista_step(c, v, xprev, (float)af, dprev, 0.f, dprev, D));
          return prox_l1(c, v, (float)(af * p->lam), x);
        }));
        ++nprox;
        CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, x, g); }));
        ++nfull;
        CS_TRY(vec_axpby(c, d, 1.f, g, -1.f, b, D));
        CS_TRY(timed(5, [&] { return objective(&f); }));
        ++n_fb;
        if (track)
          CS_TRY(vec_dist(c, x, (const float2*)p->x_ref, D, &dist_num[it], &dist_den[it]));
      }
      fobj.push_back(f);
      fprev = f;
      return CS_OK;
    };
    for (int it = 0; it < p->T; ++it) {
      const int t = p->t0 + it;
      // true gradient d = A^H (A x^t - y) = A^H A x^t - b (Alg. 1, true gradient)
      CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, x, g); }));
      ++nfull;
      CS_TRY(vec_axpby(c, d, 1.f, g, -1.f, b, D));
      if (mon) {
        if (it == 0) {
          CS_TRY(timed(5, [&] { return objective(&fprev); }));
          f0 = fprev;
        } else {
          CS_TRY(monitor(it - 1));
        }
        CS_TRY(vec_copy(c, xprev, x, D));
        CS_TRY(vec_copy(c, dprev, d, D));
      }
      // sketched model A_S^t (Alg. 1, per-iteration sketch)
      if (it > 0)
        CS_TRY(timed(3, [&] {
          return sketch_impl(c, y, p->V, p->S, p->seed, t, 0, c->smaps, nullptr);
        }));
      const float2* warm = nullptr;
      if (learned) CS_TRY(timed(4, [&] { return learned_start(warm); }));
      // K FISTA steps on 1/2||A_S(x - x^t)||^2 + <x, d> + g(x), momentum restarted
      CS_TRY(inner_fista(c, x, Ch, p->K, a, tau_l, &timed_fn, warm));
      nsk += p->K;
      nprox += p->K;
      CS_TRY(record(it));
    }
    if (mon && p->T > 0) {
      // the last iterate's gradient, for its objective
      CS_TRY(timed(0, [&] { return op_normal(c, fmaps, FC, x, g); }));
      ++nfull;
      CS_TRY(vec_axpby(c, d, 1.f, g, -1.f, b, D));
      CS_TRY(monitor(p->T - 1));
    }
    if (st) {
      st->n_warm_accepted = n_acc;
      st->n_warm_rejected = n_rej;
      st->n_fallbacks = n_fb;
      st->objective0 = f0;
      if (st->objective)
        for (size_t k = 0; k < fobj.size(); ++k) st->objective[k] = fobj[k];
    }
  }
  CS_HIP(c, hipEventRecord(ev_end, c->stream));
  CS_HIP(c, hipEventSynchronize(ev_end));
  double excluded = 0.0;
  for (int it = 0; it < p->T; ++it) {
    float ms = 0.f, md = 0.f;
    CS_HIP(c, hipEventElapsedTime(&ms, ev0, ev[it]));
    if (st && st->time_ms) st->time_ms[it] = ms - excluded;
    CS_HIP(c, hipEventElapsedTime(&md, ev[it], evd[it]));
    excluded += md;
    if (st && st->dist && track)
      st->dist[it] = std::sqrt(dist_num[it]) / std::sqrt(dist_den[it]);
  }
  float total = 0.f, prep = 0.f;
  CS_HIP(c, hipEventElapsedTime(&total, ev0, ev_end));
  CS_HIP(c, hipEventElapsedTime(&prep, ev_prep, ev0));
  if (st) {
    st->alpha = alpha;
    st->n_full_applies = nfull;
    st->n_sketch_applies = nsk;
    st->n_prox = nprox;
    st->total_ms = total - excluded;
    st->prep_ms = prep;
    double pms[6] = {0, 0, 0, 0, 0, 0};
    for (auto& ph : phases) {
      float ms = 0.f;
      CS_HIP(c, hipEventElapsedTime(&ms, ph.a, ph.b));
      pms[ph.kind] += ms;
    }
    st->ms_full_normal = pms[0];
    st->ms_sketch_normal = pms[1];
    st->ms_prox = pms[2];
    st->ms_sketch = pms[3];
    st->ms_warm = pms[4];
    st->ms_monitor = pms[5];
  }
  double chk[2];
  CS_TRY(vec_dot(c, x, x, D, chk));
  if (!std::isfinite(chk[0])) return fail(c, CS_ENUMERIC, "reconstruction produced NaN/Inf");
  return CS_OK;
}

}  // extern "C"
