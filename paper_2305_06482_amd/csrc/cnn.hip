// Learned warm start for the sketched inner solve.
//
// A small residual 3D CNN predicts the change Delta ~ x^{t+1} - x^t of one
// outer iteration of Algorithm 1 from (x^t, d^t), the current iterate and the
// full-coil gradient; the inner FISTA solve may start from x^t + Delta
// instead of x^t (the subproblem itself is unchanged, so its solution is
// too).  Layers: 4 -> 16 -> 32 -> 64 -> 2 channels, 3x3x3 convolutions with
// zero padding, ReLU after the first three.  Inputs are (re, im) of x^t / s_x
// and d^t / s_d; the output is Delta / s_o with s_o = alpha rms(d^t), the
// size of one gradient step.
//
// Every convolution is an implicit GEMM on MFMA (BF16 x BF16 -> FP32):
//   out[v][co] = sum_{tap, ci} in[v + off(tap)][ci] W[tap][ci][co] + b[co]
// with M = 16 voxels along x, N = output channels, K = 27 taps x channels.
// Activations are FP32, channel-last, channel pitch padded to 4.  The
// backward pass for the data is the same convolution with the taps flipped
// and W transposed; the weight gradient is an MFMA reduction over voxel
// chunks followed by a sum over chunks in chunk order (deterministic).
// Parameters and Adam moments are FP32; BF16 fragments of W are repacked
// after every update.
#include <cmath>
#include <cstring>

#include "cs_internal.h"

namespace cs {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kL = 4;                         // layers
constexpr int kW[kL + 1] = {4, 16, 32, 64, 2};  // channel widths
constexpr int kChunk = 4096;                  // voxels per weight-gradient partial
constexpr int kRB = 256;                      // reduction block size

__host__ __device__ inline int pad4(int c) { return (c + 3) & ~3; }

__device__ __forceinline__ short bf16r(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// ---- convolution (forward, and backward for the data) ---------------------
// in [nz][ny][nx][cinp], out [nz][ny][nx][coutp] (FP32).  B fragments
// [nk][NT][64 lanes][4]: lane l holds B[k = kb 16 + 4 (l / 16) + e][n = nt 16 +
// l % 16].  epi: 0 none, 1 bias + ReLU, 2 bias, 3 times (mask > 0).
template <int NT>
__global__ __launch_bounds__(256) void k_conv3d(const float* __restrict__ in, int cinp, int nz,
                                                int ny, int nx, const v4s* __restrict__ B,
                                                int nk, const float* __restrict__ bias,
                                                int cout, int epi,
                                                const float* __restrict__ mask,
                                                float* __restrict__ out, int coutp) {
  const int lane = threadIdx.x & 63;
  const int ntx = (nx + 15) >> 4;
  const long long tiles = (long long)ntx * ny * nz;
  const long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= tiles) return;  // whole wave
  const int tx = (int)(tile % ntx);
  const int y = (int)((tile / ntx) % ny);
  const int z = (int)(tile / ((long long)ntx * ny));
  const int m = lane & 15, g = lane >> 4;
  const int x = tx * 16 + m;
  v4f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < nk; ++kb) {
    const int k0 = kb * 16 + 4 * g;
    const int tap = k0 / cinp, ci = k0 - tap * cinp;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tap < 27 && x < nx) {
      const int zz = z + tap / 9 - 1, yy = y + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
      if ((unsigned)zz < (unsigned)nz && (unsigned)yy < (unsigned)ny &&
          (unsigned)xx < (unsigned)nx)
        a = *reinterpret_cast<const float4*>(
            in + (((long long)zz * ny + yy) * nx + xx) * cinp + ci);
    }
    const v4s av = (v4s){bf16r(a.x), bf16r(a.y), bf16r(a.z), bf16r(a.w)};
#pragma unroll
    for (int t = 0; t < NT; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, B[((long long)kb * NT + t) * 64 + lane],
                                                        acc[t], 0, 0, 0);
  }
  // D: lane holds column n = lane % 16 of rows (voxels) 4 (lane / 16) + v
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 16 + m;
    if (col >= coutp) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int xm = tx * 16 + 4 * g + v;
      if (xm >= nx) continue;
      const long long idx = (((long long)z * ny + y) * nx + xm) * coutp + col;
      float val = acc[t][v];
      if ((epi == 1 || epi == 2) && col < cout) val += bias[col];
      if (epi == 1) val = fmaxf(val, 0.f);
      if (epi == 3) val = mask[idx] > 0.f ? val : 0.f;
      out[idx] = val;
    }
  }
}

// BF16 fragments of a layer's weights W [27][cin][cout] (FP32).  Forward:
// K index k = tap pad4(cin) + ci, N index co.  Backward for the data: K index
// k = tap' pad4(cout) + co with tap' = 26 - tap, N index ci.
__global__ void k_pack_w(const float* __restrict__ W, int cin, int cout, int nk, int nt,
                         int backward, v4s* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nk * nt * 64) return;
  const int lane = (int)(i % 64);
  const int t = (int)((i / 64) % nt);
  const int kb = (int)(i / (64LL * nt));
  const int n = t * 16 + (lane & 15);
  v4s r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = kb * 16 + 4 * (lane >> 4) + e;
    float v = 0.f;
    if (!backward) {
      const int kp = pad4(cin), tap = k / kp, ci = k - tap * kp;
      if (tap < 27 && ci < cin && n < cout) v = W[((long long)tap * cin + ci) * cout + n];
    } else {
      const int kp = pad4(cout), tap = k / kp, co = k - tap * kp;
      if (tap < 27 && co < cout && n < cin) v = W[((long long)(26 - tap) * cin + n) * cout + co];
    }
    r[e] = bf16r(v);
  }
  out[i] = r;
}

// ---- weight and bias gradients ---------------------------------------------
// part[chunk][tap][cinp][coutp] = sum over the chunk's voxels v of
// in[v + off(tap)][ci] gout[v][co].  One wave per (chunk, tap, M tile, N tile).
__global__ __launch_bounds__(64) void k_conv_wgrad(const float* __restrict__ in, int cinp,
                                                   const float* __restrict__ gout, int coutp,
                                                   int nz, int ny, int nx, int mt_n, int nt_n,
                                                   float* __restrict__ part) {
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x, tap = blockIdx.y;
  const int mt = blockIdx.z % mt_n, nt = blockIdx.z / mt_n;
  const long long V = (long long)nz * ny * nx;
  const long long beg = (long long)chunk * kChunk;
  const long long end = min(V, beg + kChunk);
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int r = lane & 15, g = lane >> 4;
  const int ci = mt * 16 + r, co = nt * 16 + r;
  v4f acc = (v4f){0.f, 0.f, 0.f, 0.f};
  for (long long vb = beg; vb < end; vb += 16) {
    v4s av, bv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long long v = vb + 4 * g + e;
      float a = 0.f, b = 0.f;
      if (v < end) {
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        if (ci < cinp && (unsigned)zz < (unsigned)nz && (unsigned)yy < (unsigned)ny &&
            (unsigned)xx < (unsigned)nx)
          a = in[(((long long)zz * ny + yy) * nx + xx) * cinp + ci];
        if (co < coutp) b = gout[v * coutp + co];
      }
      av[e] = bf16r(a);
      bv[e] = bf16r(b);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
  // D: lane holds column co = nt 16 + lane % 16 of rows ci = mt 16 + 4 g + v
  if (co < coutp) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cr = mt * 16 + 4 * g + v;
      if (cr < cinp)
        part[(((long long)chunk * 27 + tap) * cinp + cr) * coutp + co] = acc[v];
    }
  }
}

// gW[tap][ci][co] = sum over chunks, in chunk order
__global__ void k_wgrad_sum(const float* __restrict__ part, int nchunk, int cin, int cout,
                            int cinp, int coutp, float* __restrict__ gW) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 27 * cin * cout) return;
  const int co = i % cout, ci = (i / cout) % cin, tap = i / (cout * cin);
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c)
    s += part[(((long long)c * 27 + tap) * cinp + ci) * coutp + co];
  gW[i] = s;
}

// gb[co] = sum_v gout[v][co]: block co, fixed strided ranges then a fixed tree
__global__ __launch_bounds__(kRB) void k_bgrad(const float* __restrict__ gout, int coutp,
                                               long long V, float* __restrict__ gb) {
  __shared__ double s[kRB];
  const int co = blockIdx.x;
  double a = 0.0;
  for (long long v = threadIdx.x; v < V; v += kRB) a += gout[v * coutp + co];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = kRB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) gb[co] = (float)s[0];
}

// ---- loss, optimiser, packing of solver data --------------------------------
// mean squared error over voxels, summed over the 2 output channels:
// gout = 2 (pred - target) / V (pitch 4), block partials of sum (pred - target)^2
__global__ __launch_bounds__(kRB) void k_mse(const float* __restrict__ pred,
                                             const float* __restrict__ target, long long V,
                                             float* __restrict__ gout, double* __restrict__ part) {
  __shared__ double s[kRB];
  const long long per = (V + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * per, end = min(V, beg + per);
  double a = 0.0;
  const float sc = 2.f / (float)V;
  for (long long v = beg + threadIdx.x; v < end; v += kRB) {
    const float e0 = pred[v * 4] - target[v * 2], e1 = pred[v * 4 + 1] - target[v * 2 + 1];
    a += (double)e0 * e0 + (double)e1 * e1;
    gout[v * 4] = sc * e0;
    gout[v * 4 + 1] = sc * e1;
    gout[v * 4 + 2] = 0.f;
    gout[v * 4 + 3] = 0.f;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = kRB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kRB) void k_sum_parts(const double* __restrict__ part, int n,
                                                   double* __restrict__ out) {
  __shared__ double s[kRB];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += kRB) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = kRB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// Adam (Kingma & Ba), bias-corrected step
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, long long n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

__global__ void k_pack_input(const float2* __restrict__ x, const float2* __restrict__ d,
                             long long D, float ix, float id, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  const float2 a = x[i], b = d[i];
  *reinterpret_cast<float4*>(out + i * 4) = make_float4(a.x * ix, a.y * ix, b.x * id, b.y * id);
}

__global__ void k_pack_target(const float2* __restrict__ xn, const float2* __restrict__ xo,
                              long long D, float inv, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  const float2 a = xn[i], b = xo[i];
  out[2 * i] = (a.x - b.x) * inv;
  out[2 * i + 1] = (a.y - b.y) * inv;
}

// z0 = x + s (pred_0, pred_1)   (pred pitch 4)
__global__ void k_apply_delta(const float2* __restrict__ x, const float* __restrict__ pred,
                              long long D, float s, float2* __restrict__ z0) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  const float2 a = x[i];
  z0[i] = make_float2(a.x + s * pred[i * 4], a.y + s * pred[i * 4 + 1]);
}

__global__ void k_copy2(const float* __restrict__ pred, long long V, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  out[2 * i] = pred[4 * i];
  out[2 * i + 1] = pred[4 * i + 1];
}

unsigned blocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// SplitMix64 (Steele, Lea & Flood) as the initialiser's generator
uint64_t sm64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

}  // namespace
}  // namespace cs

using namespace cs;

struct cs_cnn {
  hipStream_t stream = nullptr;
  long long nparam = 0;
  long long woff[kL], boff[kL];
  float* params = nullptr;  // per layer W [27][cin][cout], then b [cout]
  float* grads = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  long long step = 0;
  v4s* fwd[kL] = {};
  v4s* bwd[kL] = {};
  int fwd_nk[kL], bwd_nk[kL], fwd_nt[kL], bwd_nt[kL];
  long long cap = 0;        // voxels the activation buffers hold
  float* act[kL + 1] = {};  // act[0] input (pitch 4), act[l + 1] output of layer l
  float* gact[kL + 1] = {};
  float* wpart = nullptr;
  size_t wpart_cap = 0;
  double* dpart = nullptr;  // loss partials
  double* dsum = nullptr;
  double* host = nullptr;   // pinned readback
  // orders the network's stream and a reconstruction context's stream around
  // a warm start (they may differ): net_done is recorded on the network's
  // stream before the forward pass, ctx_done on the context's stream after
  hipEvent_t net_done = nullptr, ctx_done = nullptr;
  std::string err;
};

namespace cs {
namespace {

int cfail(cs_cnn* n, int code, const std::string& msg) {
  n->err = msg;
  return code;
}
#define CNN_HIP(n, expr)                                                               \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return cfail((n), CS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));  \
  } while (0)

int repack(cs_cnn* n, hipStream_t s) {
  for (int l = 0; l < kL; ++l) {
    const long long nf = (long long)n->fwd_nk[l] * n->fwd_nt[l] * 64;
    hipLaunchKernelGGL(k_pack_w, dim3(blocks(nf, 256)), dim3(256), 0, s, n->params + n->woff[l],
                       kW[l], kW[l + 1], n->fwd_nk[l], n->fwd_nt[l], 0, n->fwd[l]);
    const long long nb = (long long)n->bwd_nk[l] * n->bwd_nt[l] * 64;
    hipLaunchKernelGGL(k_pack_w, dim3(blocks(nb, 256)), dim3(256), 0, s, n->params + n->woff[l],
                       kW[l], kW[l + 1], n->bwd_nk[l], n->bwd_nt[l], 1, n->bwd[l]);
  }
  CNN_HIP(n, hipGetLastError());
  return CS_OK;
}

int ensure(cs_cnn* n, long long V) {
  if (V <= n->cap) return CS_OK;
  CNN_HIP(n, hipStreamSynchronize(n->stream));
  for (int l = 0; l <= kL; ++l) {
    if (n->act[l]) CNN_HIP(n, hipFree(n->act[l]));
    if (n->gact[l]) CNN_HIP(n, hipFree(n->gact[l]));
    n->act[l] = n->gact[l] = nullptr;
    const size_t bytes = sizeof(float) * (size_t)V * pad4(kW[l]);
    CNN_HIP(n, hipMalloc(&n->act[l], bytes));
    CNN_HIP(n, hipMalloc(&n->gact[l], bytes));
  }
  n->cap = V;
  return CS_OK;
}

// NT (output-channel tiles per wave) must equal the tiles the fragments B
// were packed with: 1, 2 or 4 for the widths above
bool launch_conv(hipStream_t s, int nt, const float* in, int cinp, int nz, int ny, int nx,
                 const v4s* B, int nk, const float* bias, int cout, int epi, const float* mask,
                 float* out, int coutp) {
  const long long tiles = (long long)((nx + 15) / 16) * ny * nz;
  const dim3 grid(blocks(tiles, 4)), blk(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL(k_conv3d<1>, grid, blk, 0, s, in, cinp, nz, ny, nx, B, nk, bias,
                               cout, epi, mask, out, coutp); return true;
    case 2: hipLaunchKernelGGL(k_conv3d<2>, grid, blk, 0, s, in, cinp, nz, ny, nx, B, nk, bias,
                               cout, epi, mask, out, coutp); return true;
    case 4: hipLaunchKernelGGL(k_conv3d<4>, grid, blk, 0, s, in, cinp, nz, ny, nx, B, nk, bias,
                               cout, epi, mask, out, coutp); return true;
    default: return false;
  }
}

// forward over act[0] (filled by the caller); the prediction is act[kL]
int forward(cs_cnn* n, int nz, int ny, int nx, hipStream_t s) {
  for (int l = 0; l < kL; ++l)
    if (!launch_conv(s, n->fwd_nt[l], n->act[l], pad4(kW[l]), nz, ny, nx, n->fwd[l],
                     n->fwd_nk[l], n->params + n->boff[l], kW[l + 1], l + 1 < kL ? 1 : 2,
                     nullptr, n->act[l + 1], pad4(kW[l + 1])))
      return cfail(n, CS_EINVAL, "convolution tile count");
  CNN_HIP(n, hipGetLastError());
  return CS_OK;
}

// loss and gradients for act[0] -> target (device [V][2]); gradients in n->grads
int loss_grad(cs_cnn* n, const float* target, int nz, int ny, int nx, double* loss) {
  const hipStream_t s = n->stream;
  const long long V = (long long)nz * ny * nx;
  CS_TRY(forward(n, nz, ny, nx, s));
  hipLaunchKernelGGL(k_mse, dim3(kRB), dim3(kRB), 0, s, n->act[kL], target, V, n->gact[kL],
                     n->dpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kRB), 0, s, n->dpart, kRB, n->dsum);
  const int nchunk = (int)((V + kChunk - 1) / kChunk);
  for (int l = kL - 1; l >= 0; --l) {
    const int cin = kW[l], cout = kW[l + 1], cinp = pad4(cin), coutp = pad4(cout);
    const size_t need = (size_t)nchunk * 27 * cinp * coutp;
    if (need > n->wpart_cap) {
      CNN_HIP(n, hipStreamSynchronize(s));
      if (n->wpart) CNN_HIP(n, hipFree(n->wpart));
      n->wpart = nullptr;
      CNN_HIP(n, hipMalloc(&n->wpart, sizeof(float) * need));
      n->wpart_cap = need;
    }
    const int mt_n = (cinp + 15) / 16, nt_n = (coutp + 15) / 16;
    hipLaunchKernelGGL(k_conv_wgrad, dim3(nchunk, 27, mt_n * nt_n), dim3(64), 0, s, n->act[l],
                       cinp, n->gact[l + 1], coutp, nz, ny, nx, mt_n, nt_n, n->wpart);
    hipLaunchKernelGGL(k_wgrad_sum, dim3(blocks(27LL * cin * cout, 256)), dim3(256), 0, s,
                       n->wpart, nchunk, cin, cout, cinp, coutp, n->grads + n->woff[l]);
    hipLaunchKernelGGL(k_bgrad, dim3(cout), dim3(kRB), 0, s, n->gact[l + 1], coutp, V,
                       n->grads + n->boff[l]);
    // gradient w.r.t. this layer's input, through the ReLU before it
    if (l > 0 && !launch_conv(s, n->bwd_nt[l], n->gact[l + 1], coutp, nz, ny, nx, n->bwd[l],
                              n->bwd_nk[l], nullptr, cin, 3, n->act[l], n->gact[l], cinp))
      return cfail(n, CS_EINVAL, "convolution tile count");
  }
  CNN_HIP(n, hipGetLastError());
  CNN_HIP(n, hipMemcpyAsync(n->host, n->dsum, sizeof(double), hipMemcpyDeviceToHost, s));
  CNN_HIP(n, hipStreamSynchronize(s));
  if (loss) *loss = n->host[0] / (double)V;
  return CS_OK;
}

}  // namespace

// ---- pieces used by the reconstruction --------------------------------------
int cnn_pack_input(cs_ctx* c, const float2* x, const float2* d, float sx, float sd,
                   float* out) {
  hipLaunchKernelGGL(k_pack_input, dim3(blocks(c->D, 256)), dim3(256), 0, c->stream, x, d,
                     c->D, 1.f / sx, 1.f / sd, out);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

int cnn_pack_target(cs_ctx* c, const float2* xn, const float2* xo, float so, float* out) {
  hipLaunchKernelGGL(k_pack_target, dim3(blocks(c->D, 256)), dim3(256), 0, c->stream, xn, xo,
                     c->D, 1.f / so, out);
  CS_HIP(c, hipGetLastError());
  return CS_OK;
}

// z0 = x + s_o CNN(x / s_x, d / s_d), on the context stream
int cnn_warm_start(cs_cnn* n, cs_ctx* c, const float2* x, const float2* d, float sx, float sd,
                   float so, float2* z0) {
  if (c->ndim != 3 && c->ndim != 2) return fail(c, CS_EINVAL, "CNN volume");
  const int nz = c->ndim == 3 ? c->nz : 1;
  if (ensure(n, c->D) != CS_OK) return fail(c, CS_EHIP, "CNN buffers: " + n->err);
  // the forward pass below runs on the context stream but reads the
  // parameters and fragments that training steps write on the network's
  // stream, and writes the activations those steps also use: wait for the
  // network's earlier work first, and make its later work wait for this
  const bool other = n->stream != c->stream;
  if (other) {
    CS_HIP(c, hipEventRecord(n->net_done, n->stream));
    CS_HIP(c, hipStreamWaitEvent(c->stream, n->net_done, 0));
  }
  CS_TRY(cnn_pack_input(c, x, d, sx, sd, n->act[0]));
  if (forward(n, nz, c->ny, c->nx, c->stream) != CS_OK)
    return fail(c, CS_EHIP, "CNN forward: " + n->err);
  hipLaunchKernelGGL(k_apply_delta, dim3(blocks(c->D, 256)), dim3(256), 0, c->stream, x,
                     n->act[kL], c->D, so, z0);
  CS_HIP(c, hipGetLastError());
  if (other) {
    CS_HIP(c, hipEventRecord(n->ctx_done, c->stream));
    CS_HIP(c, hipStreamWaitEvent(n->stream, n->ctx_done, 0));
  }
  return CS_OK;
}

}  // namespace cs

extern "C" {

int cs_cnn_create(void* stream, uint64_t seed, cs_cnn** out) {
  if (!out) return CS_EINVAL;
  *out = nullptr;
  auto* n = new cs_cnn();
  n->stream = (hipStream_t)stream;
  long long off = 0;
  for (int l = 0; l < kL; ++l) {
    n->woff[l] = off;
    off += 27LL * kW[l] * kW[l + 1];
    n->boff[l] = off;
    off += kW[l + 1];
    n->fwd_nk[l] = (27 * pad4(kW[l]) + 15) / 16;
    n->fwd_nt[l] = (kW[l + 1] + 15) / 16;
    n->bwd_nk[l] = (27 * pad4(kW[l + 1]) + 15) / 16;
    n->bwd_nt[l] = (kW[l] + 15) / 16;
  }
  n->nparam = off;
  // He-normal weights (std sqrt(2 / fan_in)), the last layer scaled by 0.1
  // so that the initial prediction is close to zero; zero biases
  std::vector<float> h(off, 0.f);
  uint64_t s = seed;
  for (int l = 0; l < kL; ++l) {
    const double sd = std::sqrt(2.0 / (27.0 * kW[l])) * (l + 1 == kL ? 0.1 : 1.0);
    for (long long i = 0; i < 27LL * kW[l] * kW[l + 1]; ++i) {
      const double u1 = ((sm64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      const double u2 = ((sm64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      h[n->woff[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2 * M_PI * u2));
    }
  }
  bool ok = hipMalloc(&n->params, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&n->grads, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&n->m1, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&n->m2, sizeof(float) * off) == hipSuccess &&
            hipMalloc(&n->dpart, sizeof(double) * kRB) == hipSuccess &&
            hipMalloc(&n->dsum, sizeof(double)) == hipSuccess &&
            hipHostMalloc((void**)&n->host, sizeof(double) * 2, 0) == hipSuccess &&
            hipEventCreateWithFlags(&n->net_done, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&n->ctx_done, hipEventDisableTiming) == hipSuccess;
  for (int l = 0; l < kL && ok; ++l)
    ok = hipMalloc(&n->fwd[l], sizeof(v4s) * 64 * n->fwd_nk[l] * n->fwd_nt[l]) == hipSuccess &&
         hipMalloc(&n->bwd[l], sizeof(v4s) * 64 * n->bwd_nk[l] * n->bwd_nt[l]) == hipSuccess;
  if (ok) {
    std::vector<float> zero(off, 0.f);
    ok = hipMemcpy(n->params, h.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(n->m1, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(n->m2, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(n->grads, zero.data(), sizeof(float) * off, hipMemcpyHostToDevice) ==
             hipSuccess;
  }
  if (!ok || repack(n, n->stream) != CS_OK || hipStreamSynchronize(n->stream) != hipSuccess) {
    cs_cnn_destroy(n);
    return CS_EHIP;
  }
  *out = n;
  return CS_OK;
}

void cs_cnn_destroy(cs_cnn* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  fr(n->params); fr(n->grads); fr(n->m1); fr(n->m2); fr(n->wpart); fr(n->dpart); fr(n->dsum);
  for (int l = 0; l < kL; ++l) {
    fr(n->fwd[l]);
    fr(n->bwd[l]);
  }
  for (int l = 0; l <= kL; ++l) {
    fr(n->act[l]);
    fr(n->gact[l]);
  }
  if (n->host) (void)hipHostFree(n->host);
  if (n->net_done) (void)hipEventDestroy(n->net_done);
  if (n->ctx_done) (void)hipEventDestroy(n->ctx_done);
  delete n;
}

const char* cs_cnn_last_error(const cs_cnn* n) { return n ? n->err.c_str() : ""; }

long long cs_cnn_num_params(const cs_cnn* n) { return n ? n->nparam : 0; }

int cs_cnn_get_params(cs_cnn* n, float* host, float* grad_host) {
  if (!n || (!host && !grad_host)) return CS_EINVAL;
  if (host)
    CNN_HIP(n, hipMemcpy(host, n->params, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
  if (grad_host)
    CNN_HIP(n, hipMemcpy(grad_host, n->grads, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
  return CS_OK;
}

int cs_cnn_set_params(cs_cnn* n, const float* host) {
  if (!n || !host) return CS_EINVAL;
  CNN_HIP(n, hipStreamSynchronize(n->stream));
  CNN_HIP(n, hipMemcpy(n->params, host, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
  CS_TRY(repack(n, n->stream));
  CNN_HIP(n, hipStreamSynchronize(n->stream));
  return CS_OK;
}

int cs_cnn_forward(cs_cnn* n, const float* in, int nz, int ny, int nx, float* out) {
  if (!n || !in || !out || nz < 1 || ny < 1 || nx < 1) return CS_EINVAL;
  const long long V = (long long)nz * ny * nx;
  CS_TRY(ensure(n, V));
  CNN_HIP(n, hipMemcpyAsync(n->act[0], in, sizeof(float) * 4 * V, hipMemcpyDeviceToDevice,
                            n->stream));
  CS_TRY(forward(n, nz, ny, nx, n->stream));
  hipLaunchKernelGGL(k_copy2, dim3(blocks(V, 256)), dim3(256), 0, n->stream, n->act[kL], V, out);
  CNN_HIP(n, hipGetLastError());
  return CS_OK;
}

int cs_cnn_loss_grad(cs_cnn* n, const float* in, const float* target, int nz, int ny, int nx,
                     double* loss) {
  if (!n || !in || !target || nz < 1 || ny < 1 || nx < 1) return CS_EINVAL;
  const long long V = (long long)nz * ny * nx;
  CS_TRY(ensure(n, V));
  CNN_HIP(n, hipMemcpyAsync(n->act[0], in, sizeof(float) * 4 * V, hipMemcpyDeviceToDevice,
                            n->stream));
  return loss_grad(n, target, nz, ny, nx, loss);
}

int cs_cnn_train_step(cs_cnn* n, const float* in, const float* target, int nz, int ny, int nx,
                      float lr, double* loss) {
  CS_TRY(cs_cnn_loss_grad(n, in, target, nz, ny, nx, loss));
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)n->step), bc2 = 1.f - std::pow(b2, (float)n->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(n->nparam, 256)), dim3(256), 0, n->stream, n->params,
                     n->grads, n->m1, n->m2, n->nparam, lr, b1, b2, 1e-8f, bc1, bc2);
  CNN_HIP(n, hipGetLastError());
  return repack(n, n->stream);
}

}  // extern "C"
