// Batched reconstruction of independent slices (many contexts of uneven
// sizes, coil counts and sketch sizes) and the spreading autotuner.
//
// Each slice keeps its own context and stream.  One outer iteration of
// Algorithm 1 (Sec. 2.3.4) runs, per slice, the full-coil gradient and the
// formation of the sketched maps eagerly (the sketch draw and the mixing
// fragments are prepared on the host), then the K inner FISTA iterations of
// every slice as one HIP graph: captured once with a fork onto the slice
// streams, so that the small kernels of different slices overlap on the GPU,
// and replayed for every later outer iteration with no per-kernel launch
// cost.  The graph holds only kernels (no memset nodes); it reads and writes
// fixed per-slice buffers, so a replay recomputes the same iteration on the
// current contents.
#include <chrono>
#include <cmath>
#include <cstring>

#include "cs_internal.h"

struct cs_batch {
  std::vector<cs_ctx*> ctx;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  size_t graph_nodes = 0;
  std::string err;
};

namespace cs {
namespace {

int bfail(cs_batch* b, int code, const std::string& msg) {
  b->err = msg;
  return code;
}

#define CS_BHIP(b, expr)                                                                     \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return bfail((b), CS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));        \
  } while (0)

// the context's error, prefixed with the slice index
int slice_fail(cs_batch* b, int i, int rc) {
  b->err = "slice " + std::to_string(i) + ": " + b->ctx[i]->err;
  return rc;
}

void drop_graph(cs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_nodes = 0;
}

// main stream waits for every slice stream, or every slice stream for main
int join_to_main(cs_batch* b) {
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    CS_BHIP(b, hipEventRecord(b->join[i], b->ctx[i]->stream));
    CS_BHIP(b, hipStreamWaitEvent(b->stream, b->join[i], 0));
  }
  return CS_OK;
}
int fork_from_main(cs_batch* b) {
  CS_BHIP(b, hipEventRecord(b->fork, b->stream));
  for (auto* c : b->ctx) CS_BHIP(b, hipStreamWaitEvent(c->stream, b->fork, 0));
  return CS_OK;
}

}  // namespace
}  // namespace cs

using namespace cs;

extern "C" {

int cs_batch_create(cs_ctx* const* ctxs, int n, void* stream, cs_batch** out) {
  if (!ctxs || n < 1 || !out) return CS_EINVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || (stream && ctxs[i]->stream == (hipStream_t)stream))
      return CS_EINVAL;  // the fork needs the slices off the batch stream
  auto* b = new cs_batch();
  b->ctx.assign(ctxs, ctxs + n);
  b->stream = (hipStream_t)stream;
  if (!b->stream) {
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      delete b;
      return CS_EHIP;
    }
    b->own_stream = true;
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return CS_EHIP;
  }
  b->join.resize(n, nullptr);
  for (auto& e : b->join)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto& q : b->join)
        if (q) (void)hipEventDestroy(q);
      (void)hipEventDestroy(b->fork);
      if (b->own_stream) (void)hipStreamDestroy(b->stream);
      delete b;
      return CS_EHIP;
    }
  *out = b;
  return CS_OK;
}

void cs_batch_destroy(cs_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto* c : b->ctx) (void)hipStreamSynchronize(c->stream);
  drop_graph(b);
  for (auto e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char* cs_batch_last_error(const cs_batch* b) { return b ? b->err.c_str() : ""; }

int cs_batch_recon(cs_batch* b, const void* const* y, const cs_recon_params* p,
                   void* const* x, int use_graph, cs_batch_stats* st) {
  if (!b || !y || !p || !x) return CS_EINVAL;
  const int n = (int)b->ctx.size();
  const int T = p[0].T, K = p[0].K;
  for (int i = 0; i < n; ++i) {
    cs_ctx* c = b->ctx[i];
    if (!y[i] || !x[i]) return bfail(b, CS_EINVAL, "null slice buffer");
    if (!c->have_op) return bfail(b, CS_EINVAL, "slice without an operator");
    if (p[i].mode != CS_RECON_SKETCH || p[i].reg != CS_REG_L1WAV || p[i].T != T ||
        p[i].K != K || K < 1 || T < 0)
      return bfail(b, CS_EINVAL, "every slice needs SKETCH mode and the same T and K");
    if ((p[i].C0 > 0 && p[i].C0 < c->C) || p[i].init_iters != 0 || p[i].monitor != 0)
      return bfail(b, CS_EINVAL,
                   "the batch runs Algorithm 1 on all coils, without compression, the "
                   "classical-sketch initialisation or the objective monitor");
  }
  drop_graph(b);
  for (auto* c : b->ctx) CS_BHIP(b, hipStreamSynchronize(c->stream));
  auto t_start = std::chrono::steady_clock::now();
  std::vector<float> a(n), tau_l(n);
  // set-up per slice: b = A^H y, PCA basis and first sketch, step size
  for (int i = 0; i < n; ++i) {
    cs_ctx* c = b->ctx[i];
    const cs_recon_params& q = p[i];
    const float2* yi = (const float2*)y[i];
    int rc;
    if ((rc = adjoint_all(c, c->maps, c->C, yi, c->img[0]))) return slice_fail(b, i, rc);
    c->have_b = true;
    c->b_c0 = c->C;
    if ((rc = sketch_impl(c, yi, q.V, q.S, q.seed, q.t0, 0, c->smaps, nullptr)))
      return slice_fail(b, i, rc);
    double alpha = q.step;
    if (alpha <= 0) {
      double L = 0;
      if ((rc = power_iter(c, c->smaps, q.V + q.S, q.n_pow > 0 ? q.n_pow : 30, &L)))
        return slice_fail(b, i, rc);
      alpha = 1.0 / L;
    }
    a[i] = (float)alpha;
    tau_l[i] = (float)(alpha * q.lam);
    if (st) st[i].alpha = alpha;
  }
  for (auto* c : b->ctx) CS_BHIP(b, hipStreamSynchronize(c->stream));
  auto t_loop = std::chrono::steady_clock::now();
  long long replays = 0;
  for (int it = 0; it < T; ++it) {
    // eager part: full gradient d = A^H A x^t - b and the sketched maps
    for (int i = 0; i < n; ++i) {
      cs_ctx* c = b->ctx[i];
      const cs_recon_params& q = p[i];
      float2* xi = (float2*)x[i];
      int rc;
      if ((rc = op_normal(c, c->maps, c->C, xi, c->img[5]))) return slice_fail(b, i, rc);
      if ((rc = vec_axpby(c, c->img[1], 1.f, c->img[5], -1.f, c->img[0], c->D)))
        return slice_fail(b, i, rc);
      if (it > 0 &&
          (rc = sketch_impl(c, (const float2*)y[i], q.V, q.S, q.seed, q.t0 + it, 0, c->smaps,
                            nullptr)))
        return slice_fail(b, i, rc);
    }
    if (!use_graph) {
      for (int i = 0; i < n; ++i) {
        int rc = inner_fista(b->ctx[i], (float2*)x[i], p[i].V + p[i].S, K, a[i], tau_l[i],
                             nullptr, nullptr);
        if (rc) return slice_fail(b, i, rc);
      }
      continue;
    }
    CS_TRY(join_to_main(b));
    if (!b->exec) {
      // capture the K inner iterations of every slice, forked onto the
      // slice streams
      CS_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
      int rc = fork_from_main(b);
      for (int i = 0; i < n && rc == CS_OK; ++i) {
        rc = inner_fista(b->ctx[i], (float2*)x[i], p[i].V + p[i].S, K, a[i], tau_l[i],
                         nullptr, nullptr);
        if (rc) rc = slice_fail(b, i, rc);
      }
      if (rc == CS_OK) rc = join_to_main(b);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (rc != CS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess || !g) return bfail(b, CS_EHIP, "graph capture failed");
      b->graph = g;
      CS_BHIP(b, hipGraphGetNodes(g, nullptr, &b->graph_nodes));
      CS_BHIP(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    }
    CS_BHIP(b, hipGraphLaunch(b->exec, b->stream));
    ++replays;
    CS_TRY(fork_from_main(b));
  }
  for (auto* c : b->ctx) CS_BHIP(b, hipStreamSynchronize(c->stream));
  CS_BHIP(b, hipStreamSynchronize(b->stream));
  auto t_end = std::chrono::steady_clock::now();
  for (int i = 0; i < n; ++i) {
    double chk[2];
    int rc = vec_dot(b->ctx[i], (const float2*)x[i], (const float2*)x[i], b->ctx[i]->D, chk);
    if (rc) return slice_fail(b, i, rc);
    if (!std::isfinite(chk[0])) return bfail(b, CS_ENUMERIC, "slice " + std::to_string(i) +
                                                                 ": NaN/Inf in the result");
    if (st) {
      st[i].n_full_applies = T;
      st[i].n_sketch_applies = (long long)T * K;
      st[i].wall_prep_ms = std::chrono::duration<double, std::milli>(t_loop - t_start).count();
      st[i].wall_loop_ms = std::chrono::duration<double, std::milli>(t_end - t_loop).count();
      st[i].graph_nodes = (long long)b->graph_nodes;
      st[i].graph_replays = replays;
    }
  }
  return CS_OK;
}

int cs_set_spread_cfg(cs_ctx* c, int cfg) {
  if (!c) return CS_EINVAL;
  if (cfg < 0 || cfg >= CS_SPREAD_NCFG) return fail(c, CS_EINVAL, "spread shape index");
  c->spread_cfg = cfg;
  return CS_OK;
}

int cs_set_interp_cfg(cs_ctx* c, int cfg) {
  if (!c) return CS_EINVAL;
  if (cfg < 0 || cfg >= CS_INTERP_NCFG) return fail(c, CS_EINVAL, "interpolation variant");
  c->interp_cfg = cfg;
  return CS_OK;
}

int cs_autotune_spread(cs_ctx* c, const void* maps, int ncoil, int reps, int* best,
                       double* ms) {
  if (!c || !maps || !best || ncoil < 1 || ncoil > c->C || reps < 1) return CS_EINVAL;
  if (!c->have_op) return fail(c, CS_EINVAL, "cs_set_operator has not been called");
  if (c->g.kind != CS_NONCART) {
    *best = c->spread_cfg;
    return CS_OK;
  }
  const float2* m = (const float2*)maps;
  float2* xin = c->img[8];
  float2* out = c->img[9];
  CS_TRY(vec_fill(c, xin, c->D, 1.f, 0.f));
  hipEvent_t e0, e1;
  CS_HIP(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, CS_EHIP, "event creation failed");
  }
  const int keep = c->spread_cfg;
  double best_ms = 1e30;
  int best_cfg = keep, rc = CS_OK;
  for (int cfg = 0; cfg < CS_SPREAD_NCFG && rc == CS_OK; ++cfg) {
    c->spread_cfg = cfg;
    rc = op_normal(c, m, ncoil, xin, out);  // warm-up (and LDS attribute set-up)
    if (rc) break;
    float t = 0.f;
    if (hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, CS_EHIP, "event record");
    for (int r = 0; r < reps && rc == CS_OK; ++r) rc = op_normal(c, m, ncoil, xin, out);
    if (rc == CS_OK && (hipEventRecord(e1, c->stream) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      rc = fail(c, CS_EHIP, "event timing");
    if (rc) break;
    const double per = (double)t / reps;
    if (ms) ms[cfg] = per;
    if (per < best_ms) {
      best_ms = per;
      best_cfg = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->spread_cfg = rc == CS_OK ? best_cfg : keep;
  if (rc == CS_OK) *best = best_cfg;
  return rc;
}

}  // extern "C"
