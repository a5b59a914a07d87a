// Internal declarations of the coil-sketching HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <functional>
#include <string>
#include <vector>

#include "../../include/coilsketch.h"

namespace cs {

constexpr int kCoilChunk = 16;      // coils per pass of the gridding pipeline
constexpr int kMaxFFT = 1024;       // longest axis handled by one LDS panel
constexpr int kMaxRadices = 12;

// -------------------------------------------------------------------------
// One batched, strided 1D FFT pass over an LDS panel.
//
// The array is viewed as [outer][row][column]; a work-group owns one outer
// index and Wt consecutive columns, loads the n_in rows into LDS (zero
// filling the others when the axis is zero-padded), runs the mixed-radix
// Stockham FFT along the rows, optionally multiplies by a sampling mask (and
// transforms back), and stores n_out rows.  Columns index (pixel p, coil c)
// pairs as p * cb + c; a buffer with coil leading dimension ldc and coil
// offset c0 keeps element (p, c) at p * ldc + c0 + c.
// -------------------------------------------------------------------------
enum { PRO_GRID = 0, PRO_IMAGE = 1 };
enum { EPI_GRID = 0, EPI_IMAGE = 1 };
enum { MID_NONE = 0, MID_MASK_IFFT = 1, MID_MASK = 2 };

struct PassArgs {
  int L;                 // FFT length
  int n_in, n_out;       // rows loaded / stored
  int pad_in, pad_out;   // 1: image row t <-> FFT row (t - n/2) mod L
  int dir;               // -1 forward (e^{-i}), +1 inverse (unnormalised)
  int nrad;
  int rad[kMaxRadices];
  const float2* tw;      // [L] e^{-2 pi i k / L}
  int Wt;                // panel width (columns per work-group)
  long long nblk;        // column blocks per outer index
  long long inner;       // columns per outer index
  int cb;                // coils per pixel in the column space
  // grid source / destination
  const float2* src; long long src_os, src_rs; int src_ldc, src_c0;
  float2* dst; long long dst_os, dst_rs; int dst_ldc, dst_c0;
  // masks (uint8): value at outer * mask_os + row * mask_rs
  int mid; int premask;
  const uint8_t* mask; long long mask_os, mask_rs;
  // image prologue / epilogue: pixel (t, p) at t * P + p
  int prologue, epilogue, accumulate;
  const float2* img; float2* img_out; long long P;
  const float2* maps; int maps_ldc, maps_c0;
  const float* da;       // [n] per-row scale along the pass axis
  const float* dp;       // [P] per-pixel scale of the other axes
  int xcd;               // 1: each XCD takes a contiguous range of panels
  // 1: the panel is loaded (stored) as pairs of adjacent columns, 16 bytes
  // per thread and row (grid source / destination with contiguous columns)
  int vec_in, vec_out;
  int vec_img;  // the image prologue on coil pairs of one pixel
  int sum_rows;  // coil-sum epilogue: one thread per (row, pixel)
};

// Work-groups are dealt to the 8 XCDs in turn (group b to XCD b mod 8), and
// each XCD has an L2 of its own.  This order gives XCD x a contiguous range
// of the logical groups instead, so that groups whose data are neighbours in
// memory (sharing cache lines) run on the same L2.  A bijection on [0, G).
__device__ __forceinline__ long long xcd_contiguous(long long b, long long G) {
  const long long q = G >> 3, r = G & 7, x = b & 7, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Sample record of the sorted non-Cartesian trajectory (64 bytes): first tap
// relative to the tile's origin (x | y << 8 | z << 16), density weight w and
// sqrt(w), index in the caller's order, and the four kernel weights per axis.
struct SampleRec {
  int key;
  float w, sw;
  int orig;
  float wx[4], wy[4], wz[4];
};

// A work item of the gridding kernels: samples kbeg .. kend (sorted order) of
// one tile; slot = its partial tile (items of tile t hold slots item_off[t] ..
// item_off[t + 1]); voff = the offset of its values in its item group.
struct GridItem {
  int tile, kbeg, kend, slot, voff, pad0, pad1, pad2;
};


// samples per item group of the normal operator by default (its values stay
// on chip between the interpolation and the spreading)
constexpr long long kGroupSamples = 1LL << 40;

struct FFTPlan {
  int L = 0;
  int nrad = 0;
  int rad[kMaxRadices] = {0};
  float2* tw = nullptr;  // device
};

}  // namespace cs

struct cs_ctx {
  cs_geom g{};
  hipStream_t stream = nullptr;
  std::string err;

  // normalised 3D geometry (2D: nz = mz = 1)
  int ndim = 2;
  int nz = 1, ny = 1, nx = 1;
  int mz = 1, my = 1, mx = 1;
  long long D = 0, M = 0, N = 0;
  int C = 0;
  float beta = 0.f;

  std::map<int, cs::FFTPlan> plans;
  // FFT pass panels: pixels per panel of an image pass (all coils of each)
  // and columns per panel of a grid pass (CS_FFT_PIX / CS_FFT_COLS)
  int fft_pix = 1, fft_cols = 16;
  int fft_pro_cols = 16;  // > 0: image-prologue passes in panels of this many columns
  int fft_vec_img = 1;    // image prologue loads maps as coil pairs
  int fft_sum_rows = 1;   // coil-sum epilogue over all threads of a panel
  int fft_vec = 1;  // paired-column loads and stores in the grid passes
  int grid_vec = 1;  // paired-coil accesses in the interpolation and merge
  int fft_xcd = 1;                // XCD-contiguous panel order in the FFT passes
  int grid_xcd = 1;               // gridding: an item's coil groups on one XCD
  int merge_xcd = 0;              // merge: each XCD a contiguous range of tiles

  // operator
  const float2* maps = nullptr;   // borrowed [D][C]
  bool have_op = false;
  uint8_t* mask = nullptr;        // Cartesian [D]
  bool mask1d = false;            // mask constant along x: only y-FFTs needed
  float* da[3] = {nullptr, nullptr, nullptr};  // per-axis scale tables
  float* dp_z = nullptr;          // [ny*nx] per-pixel table for a z pass
  float* dp_y = nullptr;          // [nx] per-pixel table for a y pass (2D)
  float* da_y1d = nullptr;        // [ny] 1/sqrt(ny): unitary y-only FFT pair
  float* ones = nullptr;          // [max(n)] ones

  // non-Cartesian
  cs::SampleRec* rec = nullptr;   // [N] sorted sample records
  float* dcf_orig = nullptr;      // [N] caller order (nullptr: w = 1)
  int tile[3] = {1, 1, 1};        // spread tile size (tz, ty, tx)
  int ntile[3] = {1, 1, 1};
  long long ntiles = 0;
  cs::GridItem* gitems = nullptr; // work items, grouped (group g: group_off[g] .. [g + 1])
  std::vector<int> group_off;
  long long n_items = 0;
  int* item_off = nullptr;        // [ntiles + 1]: slots of tile t are item_off[t]..[t+1]
  float2* partial = nullptr;      // halo'd partial tile of every slot
  size_t partial_elems = 0;       // float2 capacity of `partial`
  int spread_cfg = 0;             // spread work-group shape (see launch_spread)
  int interp_cfg = 1;             // interpolation: 0 per-sample gather, 1/2 LDS tiles
  int sketch_dist = 0;            // CS_SKETCH_RADEMACHER or CS_SKETCH_GAUSSIAN

  // work buffers
  bool ws_external = false;       // carved from the caller's workspace (not freed here)
  float2* gridA = nullptr;        // M * kCoilChunk
  float2* gridB = nullptr;
  float2* vbuf = nullptr;         // sample values of the largest item group (kCoilChunk coils)
  long long vbuf_pad = 0;         // extra coils allocated past its last row
  std::vector<float2*> img;       // D-sized scratch images
  double* red = nullptr;          // reduction partials
  double* red_out = nullptr;      // final reduction values (device)
  double* host_red = nullptr;     // pinned host copy
  float2* tvu = nullptr;          // [ndim][D] PDHG dual variable of the TV term
  float2* ysk = nullptr;          // [N][C^] sketched data of the classical initialisation
  size_t ysk_elems = 0;           // (allocated on its first use)
  float2* cmaps = nullptr;        // [D][C0] compressed virtual maps (initial compression)
  size_t cmaps_elems = 0;
  float2* ycmp = nullptr;         // [N][C0] compressed data
  size_t ycmp_elems = 0;
  int c0_active = 0;              // > 0 inside a compressed reconstruction
  int b_c0 = 0;                   // coil count b = A^H y was formed with

  // sketch cache
  bool have_U = false;
  std::vector<double> U;          // C*C complex (re, im) row-major
  std::vector<double> lam;
  float2* vmaps = nullptr;        // [D][C] virtual maps U^H c
  unsigned long long vmaps_gen = 1;   // bumped whenever vmaps is recomputed
  // injected random block of the sketch (cs_set_sketch): [S][C - V] as applied
  std::vector<double> inj_R;
  int inj_V = -1, inj_S = -1;
  // layout of the V identity rows last copied into smaps (from vmaps of
  // generation vrows_gen, V rows of a Ch-coil stack)
  unsigned long long vrows_gen = 0;
  int vrows_V = -1, vrows_Ch = -1;
  double* cov_part = nullptr;     // covariance partials
  double* cov = nullptr;          // [C][C] complex double
  double* eig_dev = nullptr;      // U and lambda from the eigensolver
  void* mixB = nullptr;           // packed bf16 B fragments for coil mixing
  void* mix_scratch = nullptr;    // this device's static fragment scratch (no-alloc mixing)
  size_t mixB_bytes = 0;
  // pinned staging ring for the fragments' host-to-device copies; the event
  // of a slot marks its last copy, so a slot is rewritten only after it
  static constexpr int kStage = 4;
  void* stage[kStage] = {};
  size_t stage_bytes[kStage] = {};
  hipEvent_t stage_ev[kStage] = {};
  int stage_next = 0;

  // wavelet work
  float2* wav1 = nullptr;
  float2* wav2 = nullptr;

  // recon
  bool have_b = false;
  float2* smaps = nullptr;        // [D][C] sketched maps of the current t

  // per-kernel event timing
  struct ProfRec {
    int kind;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[CS_NKERNELS] = {0};
  long long prof_cnt[CS_NKERNELS] = {0};
};

namespace cs {

// error helpers
int fail(cs_ctx* c, int code, const std::string& msg);
#define CS_HIP(ctx, expr)                                                   \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess)                                                   \
      return ::cs::fail((ctx), CS_EHIP,                                     \
                        std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)
#define CS_TRY(expr)            \
  do {                          \
    int _r = (expr);            \
    if (_r != CS_OK) return _r; \
  } while (0)

// kernel kinds for event timing (see cs_profile_read)
enum {
  K_PASS = 0, K_INTERP, K_SPREAD, K_GATHER, K_WAVELET, K_SOFT, K_VEC, K_REDUCE,
  K_COV, K_EIG, K_MIX, K_MERGE
};
void prof_begin(cs_ctx* c, int kind);
void prof_end(cs_ctx* c);
#define CS_KLAUNCH(ctx, kind, ...)     \
  do {                                 \
    ::cs::prof_begin((ctx), (kind));   \
    hipLaunchKernelGGL(__VA_ARGS__);   \
    ::cs::prof_end((ctx));             \
  } while (0)

// fft_pass.hip
int get_plan(cs_ctx* c, int L, const FFTPlan** out);
int launch_pass(cs_ctx* c, PassArgs& a, long long n_outer);
void fill_plan(PassArgs& a, const FFTPlan* p);

// grid.hip (cb <= kCoilChunk coils per call)
int setup_noncart(cs_ctx* c, const float* coords, const float* dcf);
// out_grid = spread(w * interp(grid)): the gridding stage of the normal operator
int grid_normal(cs_ctx* c, const float2* grid, int cb, float2* out_grid);
// y[caller order][c0 + j] = sqrt(w) interp(grid)_j
int grid_interp(cs_ctx* c, const float2* grid, int cb, float2* y, int ldc, int c0);
// out_grid = spread(sqrt(w) y[.][c0 + j])
int grid_spread_data(cs_ctx* c, const float2* y, int ldc, int c0, int cb, float2* out_grid);
enum { W_NONE = 0, W_SQRT = 1, W_FULL = 2 };
double kb_i0(double x);
double kb_ft(double nu, double W, double beta);

// vec.hip
int vec_fill(cs_ctx* c, float2* x, long long n, float re, float im);
int vec_axpby(cs_ctx* c, float2* out, float a, const float2* x, float b,
              const float2* y, long long n);
int vec_copy(cs_ctx* c, float2* out, const float2* x, long long n);
int vec_dot(cs_ctx* c, const float2* a, const float2* b, long long n,
            double out[2]);
int vec_fista_step(cs_ctx* c, float2* v, const float2* z, float alpha,
                   const float2* g1, float s2, const float2* g2, long long n);
int vec_momentum(cs_ctx* c, float2* z, float2* x, const float2* xn, float beta,
                 long long n);
int vec_dist(cs_ctx* c, const float2* a, const float2* b, long long n,
             double* num, double* den);
int vec_abs_sum(cs_ctx* c, const float2* a, long long n, double* out);

// wavelet.hip
int wavelet_init(cs_ctx* c);
int dwt_fwd(cs_ctx* c, const float2* x, float2* coef);
int dwt_inv(cs_ctx* c, const float2* coef, float2* x);
int prox_l1(cs_ctx* c, const float2* v, float tau, float2* out);

// sketch.hip
int covariance_eig(cs_ctx* c, const float2* y);
int coil_mix(cs_ctx* c, const float2* in, int in_ldc, int in_c0, int cin,
             const double* M, int cout, float2* out, int out_ldc, int out_c0,
             float out_scale);
// the same over `rows` rows (data [N][.] instead of maps [D][.])
int coil_mix_rows(cs_ctx* c, long long rows, const float2* in, int in_ldc, int in_c0, int cin,
                  const double* M, int cout, float2* out, int out_ldc, int out_c0,
                  float out_scale);

// allocation-free coil mixing (M device complex128 [cout][cin]); the
// fragments go to a static per-device scratch whose address mix_scratch_init
// looks up once per device
int mix_scratch_init(cs_ctx* c);
int coil_mix_reserve(cs_ctx* c);
int coil_mix_noalloc(cs_ctx* c, const float2* in, int cin, const void* M, int cout,
                     float2* out);

// operators and solver pieces (api.hip)
int op_normal(cs_ctx* c, const float2* maps, int ncoil, const float2* x,
              float2* out);
int adjoint_all(cs_ctx* c, const float2* maps, int ncoil, const float2* y, float2* x);
int power_iter(cs_ctx* c, const float2* maps, int ncoil, int n_iter, double* L);
int sketch_impl(cs_ctx* c, const float2* y, int V, int S, uint64_t seed, int t, int refresh,
                float2* smaps, std::vector<int8_t>* signs_out);
int inner_fista(cs_ctx* c, float2* x, int Ch, int K, float a, float tau_l,
                const std::function<int(int, const std::function<int()>&)>* timed,
                const float2* start);
// PDHG updates of the l1-TV regularizer: u <- clip(u + sigma T xbar, lam)
// (u holds ndim components of D), v = x - tau T^H u
int tv_dual_step(cs_ctx* c, float2* u, const float2* xbar, float sigma, float lam);
int tv_primal_step(cs_ctx* c, float2* v, const float2* x, const float2* u, float tau);
// K CG iterations on (A^H A + lam I) u = rhs (r holds rhs on entry)
int cg_solve(cs_ctx* c, const float2* maps, int ncoil, float lam, float2* u, bool u_zero,
             float2* r, float2* p, float2* q, int K, int kind,
             const std::function<int(int, const std::function<int()>&)>* timed,
             long long* napplies);

// cnn.hip: learned warm start
int cnn_pack_input(cs_ctx* c, const float2* x, const float2* d, float sx, float sd,
                   float* out);
int cnn_pack_target(cs_ctx* c, const float2* xn, const float2* xo, float so, float* out);
int cnn_warm_start(cs_cnn* n, cs_ctx* c, const float2* x, const float2* d, float sx, float sd,
                   float so, float2* z0);
int warm_scales(cs_ctx* c, const float2* x, const float2* d, double alpha, double* sx,
                double* sd, double* so);

}  // namespace cs
