/*
 * coilsketch.h -- C ABI of the MI355X (gfx950) coil-sketching library.
 *
 * The library applies the multi-coil SENSE operator of Oscanoa et al.,
 * "Coil Sketching for computationally-efficient MR iterative reconstruction"
 * (Sec. 2.1, Eqs. 1-2 and 5), its adjoint and normal operator, builds the
 * structured coil sketch of Sec. 2.3.2-2.3.3 (Eqs. 11-13), and runs the
 * reconstruction of Algorithm 1 (Sec. 2.3.4) with FISTA inner solves and the
 * l1-wavelet regularizer of Sec. 2.1.1.  Every step runs in HIP kernels.
 *
 * General rules
 *  - Every array argument marked "device" is a device pointer owned by the
 *    caller; it must stay valid until the call's work on the context stream
 *    has finished.  Host pointers are marked "host".
 *  - Complex data is complex64: interleaved (re, im) float32.
 *  - Images are row-major with the last axis fastest: [nz][ny][nx] (3D) or
 *    [ny][nx] (2D).  For the non-Cartesian operator the image index i along
 *    an axis of length n has the centred coordinate i - n/2.
 *  - Coil stacks are pixel-major with the coil index fastest: maps [D][C],
 *    data [N][C].  Cartesian data is zero-filled on the full grid (N = D),
 *    in the non-centred FFT layout (DC at index 0).
 *  - Non-Cartesian coordinates are float32 [N][ndim] in cycles/FOV, column 0
 *    the x (fastest image axis) frequency, each within [-n_a/2, n_a/2).
 *  - All calls are asynchronous on the context's stream unless stated.
 *  - Return codes: CS_OK (0), CS_EINVAL (-1: null pointer, bad size, V+S > C,
 *    unsupported FFT length), CS_EUNSUPPORTED (-2), CS_EHIP (-3: a HIP runtime
 *    error), CS_ENUMERIC (-4: NaN or divergence).  cs_last_error() gives a
 *    message.  No exception crosses the ABI.
 *  - A context is bound to one stream and is not thread-safe.  It allocates
 *    its working memory in cs_create() (or takes it from the caller's
 *    workspace, cs_create_ws) and cs_set_operator(), and frees it in
 *    cs_destroy().  sense_apply, sense_adjoint, normal_apply, sketch_build,
 *    the building blocks and recon_run's default path allocate nothing; the
 *    exceptions are named where they apply (recon_run's initial compression
 *    and classical-sketch initialisation buffers, and the CNN's activations,
 *    on first use, unless cs_reserve_recon made them).
 */
#ifndef COILSKETCH_H
#define COILSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_ctx cs_ctx;

enum {
  CS_OK = 0,
  CS_EINVAL = -1,
  CS_EUNSUPPORTED = -2,
  CS_EHIP = -3,
  CS_ENUMERIC = -4
};

enum { CS_CART = 0, CS_NONCART = 1 };

/* Geometry of one operator (Sec. 2.1: image x in C^D, C channels, N samples). */
typedef struct {
  int ndim;          /* 2 or 3 */
  int n[3];          /* image size per axis, slowest first: {nz, ny, nx} or {ny, nx, 0} */
  int ncoil;         /* C: coils of the full operator */
  int kind;          /* CS_CART (F~ = U F~_u) or CS_NONCART (F~ = F~_n, NUFFT) */
  long long nsamp;   /* N: samples per coil (non-Cartesian); ignored for Cartesian */
  float sigma;       /* NUFFT grid oversampling (e.g. 1.25); m_a = round(sigma n_a) */
  int kwidth;        /* Kaiser-Bessel width in grid cells; only 4 is supported */
  float beta;        /* KB shape; 0 selects Beatty's formula */
  int wav_levels;    /* levels of the db4 transform (image sizes divisible by 2^levels) */
} cs_geom;

/* Create a context for geometry g on HIP stream `stream` (a hipStream_t, or
 * NULL for the default stream).  On success *out holds the context. */
int cs_create(const cs_geom* g, void* stream, cs_ctx** out);

/* Device bytes of the work buffers a context for geometry g needs (grids of
 * the FFT passes, sample values, images, reductions, sketch and wavelet
 * buffers), for a caller who provides them through cs_create_ws.  Validates
 * g as cs_create does; no device work. */
int cs_workspace_size(const cs_geom* g, size_t* bytes);

/* cs_create with a caller-owned workspace: `workspace` is device memory of at
 * least cs_workspace_size(g) bytes at a 256-byte boundary (a torch buffer,
 * say) that must stay valid until cs_destroy, which does not free it
 * (CS_EINVAL if it is smaller or misaligned).  The small per-axis tables, the
 * FFT twiddles and the coil-mixing fragment buffers are still allocated
 * here, and cs_set_operator still allocates the trajectory's sorted records,
 * work items and partial tiles (their sizes depend on the binning). */
int cs_create_ws(const cs_geom* g, void* workspace, size_t ws_bytes, void* stream,
                 cs_ctx** out);

/* Destroy a context and free its device memory (synchronises its stream). */
void cs_destroy(cs_ctx* ctx);

/* Message for the last error on ctx (or the last failed cs_create if ctx is
 * NULL).  The string is owned by the library. */
const char* cs_last_error(const cs_ctx* ctx);

/* Bind the full-coil operator.  maps: device [D][C] complex64, borrowed (must
 * outlive the context's use of it).  Cartesian: mask device uint8 [D]
 * (non-centred), coords/dcf NULL.  Non-Cartesian: coords device float32
 * [N][ndim], dcf device float32 [N] (may be NULL for w = 1), mask NULL; the
 * coordinates are copied, binned and sorted here (synchronous).  Sec. 2.1:
 * A = W^1/2 F C, y = W^1/2 k. */
int cs_set_operator(cs_ctx* ctx, const void* maps, const uint8_t* mask,
                    const float* coords, const float* dcf);

/* y = W^1/2 F (c_c * x) for the ncoil maps given (Eq. 5).  maps device
 * [D][ncoil], x device [D], y device [N][ncoil] (overwritten; samples in the
 * caller's order). */
int sense_apply(cs_ctx* ctx, const void* maps, int ncoil, const void* x, void* y);

/* x = sum_c conj(c_c) * F^H W^1/2 y_c, the adjoint of sense_apply.  y device
 * [N][ncoil], x device [D] (overwritten). */
int sense_adjoint(cs_ctx* ctx, const void* maps, int ncoil, const void* y, void* x);

/* out = sum_c conj(c_c) * F^H W F (c_c * x) = A^H A x for the ncoil maps
 * given: the full set (A) or a sketched set (A_S^t, Eq. 12).  x, out device
 * [D]; they must not alias. */
int normal_apply(cs_ctx* ctx, const void* maps, int ncoil, const void* x, void* out);

/* Structured sketch of Sec. 2.3.2-2.3.3.  On the first call after
 * cs_set_operator (or when `refresh` is non-zero) the coil covariance
 * R = sum_i k_i k_i^H of the raw samples k_i = y_i / sqrt(w_i) is accumulated
 * in FP64, R = U diag(lambda) U^H is found by a FP64 Jacobi eigensolver
 * (lambda descending; each eigenvector's largest-magnitude entry made real
 * positive), and the virtual maps c' = U^H c are formed and cached.  Each call
 * then draws the Rademacher block S~_S^t in {+1,-1}^{S x (C-V)} from
 * SplitMix64(seed) at counter (t << 32 | a (C-V) + b) + 1 (sign = top bit) and
 * writes the V + S sketched maps c^ = [c'_1..V ; (S~_S^t / sqrt(S)) c'_V+1..C].
 *   y       device [N][C] data (used for the covariance only)
 *   smaps   device [D][V+S] output
 *   eig     host [C] float64 (may be NULL): lambda
 *   U_out   host [C][C] complex128 row-major, column j = eigenvector j (may be NULL)
 *   signs   host [S][C-V] int8 (may be NULL): the Rademacher draw (left
 *           untouched under the Gaussian distribution).  Synchronises when
 *           any host output is requested.
 * Requires V >= 0, S >= 0 and 0 < V + S <= C.  S = 0 with V < C keeps only
 * the V high-energy virtual coils (coil compression inside the subproblem;
 * Sec. 3.2 reports that Algorithm 1 then diverges).  The random block's
 * distribution is set per context by cs_set_sketch_dist. */
int sketch_build(cs_ctx* ctx, const void* y, int V, int S, uint64_t seed, int t,
                 int refresh, void* smaps, double* eig, double* U_out,
                 int8_t* signs);

/* Inject the PCA basis instead of computing it from the data (Sec. 2.3.3
 * fixes U only up to the phase of each eigenvector): U host complex128
 * [C][C] row-major with column j the eigenvector of virtual coil j
 * (c'_j = sum_c conj(U[c][j]) c_c), lam host [C] float64 or NULL.  Forms and
 * caches the virtual maps (asynchronous); later sketch_build and recon_run
 * calls use them until cs_set_operator or a sketch_build with refresh. */
int cs_set_basis(cs_ctx* ctx, const double* U, const double* lam);

/* Inject the random block of the sketching matrix (Eq. 11, S~_S): R host
 * float64 [S][C - V] row-major, taken as given (any 1/sqrt(S) scale
 * included), so the sketched coils are c^_{V+a} = sum_b R[a][b] c'_{V+b}.
 * Every later sketch_build and recon_run with this V and S on all C coils
 * uses it at every outer iteration instead of the seeded draw (and reports
 * no signs); R = NULL returns to the draw.  Requires V >= 0, S >= 1,
 * V + S <= C, V < C. */
int cs_set_sketch(cs_ctx* ctx, int V, int S, const double* R);

/* Distribution of the random block (Sec. 3.2): Rademacher (the default) or
 * Gaussian with variance 1/S (values / sqrt(S) with unit-variance values;
 * E[S~^T S~] = I for both).  Gaussian entry e = a (C-V) + b of outer
 * iteration t: SplitMix64(seed) outputs n1 = c + 1, n2 = c + 2 with
 * c = (t << 32) | 2e, u1 = ((z1 >> 11) + 1) 2^-53, u2 = (z2 >> 11) 2^-53 and
 * value sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller).  Applies to later
 * sketch_build and recon_run calls on this context. */
enum { CS_SKETCH_RADEMACHER = 0, CS_SKETCH_GAUSSIAN = 1 };
int cs_set_sketch_dist(cs_ctx* ctx, int dist);

/* Recon modes */
enum { CS_RECON_FULL = 0, CS_RECON_SKETCH = 1, CS_RECON_SKETCH_LEARNED = 2 };
/* Regularizers (Sec. 2.1): l1-wavelet g = lambda ||Psi x||_1, solved with
 * FISTA; l2 (Tikhonov) g = lambda/2 ||x||^2, solved with conjugate
 * gradients; l1 total variation g = lambda ||T x||_1 (T the periodic
 * first-order differences, every component's complex modulus), solved with
 * PDHG whose data-consistency step is a CG solve */
enum { CS_REG_L1WAV = 0, CS_REG_L2 = 1, CS_REG_TV = 2 };

typedef struct cs_cnn cs_cnn;

typedef struct {
  int mode;          /* CS_RECON_FULL: plain solver; CS_RECON_SKETCH: Algorithm 1 */
  float lam;         /* regularization weight lambda */
  int T;             /* FULL: solver iterations; SKETCH: outer iterations */
  int K;             /* SKETCH: inner solver iterations per subproblem */
  int V, S;          /* sketch design (Sec. 2.3.3) */
  uint64_t seed;     /* sketch seed */
  int t0;            /* first outer index (resume: x_inout holds x^{t0}) */
  double step;       /* FISTA step alpha; <= 0 selects 1/L from the power
                        iteration on the first subproblem (Sec. 3.3.1) */
  int n_pow;         /* power-iteration count (default 30) */
  int reuse_b;       /* non-zero: reuse b = A^H y from the previous call */
  const void* x_ref; /* device [D] or NULL: per-iteration distance reference */
  cs_cnn* cnn;       /* CS_RECON_SKETCH_LEARNED: the warm-start network (borrowed) */
  int reg;           /* CS_REG_L1WAV (FISTA, the default), CS_REG_L2 (CG) or
                        CS_REG_TV (PDHG); l2 and TV: FULL and SKETCH modes only */
  int n_cg;          /* CS_REG_TV: CG iterations per PDHG data-consistency step
                        (<= 0 selects 5) */
  int init_iters;    /* SKETCH / SKETCH_LEARNED with l1-wavelet: > 0 runs Alg. 1's
                        classical-sketch initialisation, x^1 = argmin
                        1/2 ||S^0 A x - S^0 y||^2 + g(x) with the sketch of
                        t = 0 on maps and data (S~^0 U^H y per sample), by this
                        many FISTA iterations from x^{t0}; the sketched data
                        buffer ([N][V+S]) is allocated on its first use */
  int C0;            /* Alg. 1's initial coil compression: 0 < C0 < C rotates the
                        model and the data onto the PCA virtual coils and keeps
                        the first C0 (the true gradient and b use them, the
                        sketches draw over them: V + S <= C0); 0 or >= C keeps
                        every coil.  Compressed maps [D][C0] and data [N][C0]
                        are allocated on first use */
  int monitor;       /* SKETCH / SKETCH_LEARNED with l1-wavelet (no counterpart in
                        the paper): non-zero evaluates the FP64 objective
                        F(x) = 1/2 ||A x - y||^2 + lambda ||Psi x||_1 (Eqs. 3-4,
                        as 1/2 <x, A^H A x> - Re <x, A^H y> + 1/2 ||y||^2 +
                        lambda ||Psi x||_1 from the true gradient's apply) of
                        x^{t0} and of every outer iterate.  An iterate whose F
                        is not finite or exceeds F(x^t) + mon_tol |F(x^t)| is
                        replaced by one full-coil proximal-gradient step from
                        x^t, x^{t+1} = prox_{lambda / L}(x^t - d^t / L), with L
                        from the power iteration on the full operator (run at
                        the first fallback); the run then continues from it.
                        Costs one more full-coil apply after the last outer
                        iteration, two FP64 dot products and a wavelet
                        transform per outer iteration */
  double mon_tol;    /* the monitor's relative increase tolerance (>= 0) */
} cs_recon_params;

typedef struct {
  /* host arrays of length >= T, filled when non-NULL */
  double* dist;      /* ||x^t - x_ref|| / ||x_ref|| (FP64) after each iteration */
  double* time_ms;   /* GPU time since the start of the loop, per iteration */
  /* scalar outputs */
  double alpha;      /* step used */
  long long n_full_applies;    /* full-coil normal applies */
  long long n_sketch_applies;  /* sketched normal applies */
  long long n_prox;            /* wavelet prox evaluations */
  double total_ms;   /* GPU time of the whole call */
  /* GPU time (HIP events on the context stream) spent in each phase of the
   * iterations: full-coil normal applies, sketched normal applies, wavelet
   * prox, and forming the sketched maps */
  double ms_full_normal, ms_sketch_normal, ms_prox, ms_sketch;
  /* GPU time before the first iteration: b = A^H y (unless reused), the PCA
   * basis and first sketch (SKETCH), and the power iteration (step <= 0) */
  double prep_ms;
  /* SKETCH_LEARNED: outer iterations whose warm start was accepted / fell
   * back to the plain start, and the GPU time of the warm-start decisions */
  long long n_warm_accepted, n_warm_rejected;
  double ms_warm;
  /* monitor (cs_recon_params.monitor): host array of length >= T filled when
   * non-NULL with F(x^{t0+it+1}) of the accepted iterate after outer
   * iteration it; F of the iterate the outer loop starts from (x^{t0}, or
   * the classical-sketch initialisation's result when it runs); the outer
   * iterations replaced by the full-coil step; and the GPU time of the
   * objective evaluations and fallbacks */
  double* objective;
  double objective0;
  long long n_fallbacks;
  double ms_monitor;
} cs_recon_stats;

/* Allocate recon_run's optional buffers now, so that recon_run allocates
 * nothing: the compressed maps and data of an initial compression to up to
 * C0 virtual coils ([D][C0] and [N][C0]) and the sketched data of the
 * classical-sketch initialisation with up to init_coils = V + S coils
 * ([N][init_coils]); 0 skips either.  Synchronous (hipMalloc). */
int cs_reserve_recon(cs_ctx* ctx, int C0, int init_coils);

/* Reconstruction (Algorithm 1 or the plain solver) of x from data y on the
 * operator bound by cs_set_operator.  y device [N][C]; x_inout device [D]:
 * x^{t0} on entry, the result on exit.  The PCA basis comes from the data of
 * the first sketch after cs_set_operator and stays cached for later calls
 * (sketch_build with refresh recomputes it from new data).  With CS_REG_L2, FULL runs T CG
 * iterations on (A^H A + lambda I) x = A^H y from x^{t0}, and SKETCH runs
 * Algorithm 1 whose subproblem (Eq. 10 with g = lambda/2 ||x||^2) is the
 * linear system (A_S^H A_S + lambda I) u = -(d^t + lambda x^t), solved by K
 * CG iterations from u = 0, x^{t+1} = x^t + u; no step size is needed (alpha
 * is reported as 0) and CG scalars are FP64 reductions.  With CS_REG_TV,
 * FULL runs T PDHG iterations (Chambolle-Pock, theta = 1,
 * tau = sigma = 1/sqrt(4 ndim), dual variable starting at 0):
 *   u <- clip(u + sigma T xbar, lambda),  v = x - tau T^H u,
 *   x <- solution of (A^H A + I/tau) x = A^H y + v/tau (n_cg CG iterations
 *        warm-started at x),  xbar = 2 x_new - x_old;
 * SKETCH runs Algorithm 1 with K such PDHG iterations per subproblem, whose
 * data-consistency system is (A_S^H A_S + I/tau) x = A_S^H A_S x^t - d^t + v/tau.
 * CS_RECON_SKETCH_LEARNED runs Algorithm 1 with each subproblem's FISTA
 * started at
 * z0 = x^t + s_o CNN(x^t / s_x, d^t / s_d) (s_d = rms(d^t), s_o = alpha s_d,
 * s_x = rms(x^t) or s_o while x^t = 0) when the FP64 subproblem objective
 * at z0 is no larger than at x^t, else at x^t (the fallback); the
 * subproblems, hence the method's fixed point, are unchanged.  The monitor
 * (p->monitor) is for the l1-wavelet SKETCH and SKETCH_LEARNED modes only:
 * CS_EINVAL with another mode or regularizer, or with mon_tol < 0 or NaN.
 * Errors also: CS_ENUMERIC when the result holds NaN/Inf.  Synchronous. */
int recon_run(cs_ctx* ctx, const void* y, const cs_recon_params* p,
              void* x_inout, cs_recon_stats* st);

/* ---- learned warm start (no counterpart in the paper) ------------------------
 * A residual 3D CNN, 4 -> 16 -> 32 -> 64 -> 2 channels, 3x3x3 convolutions
 * (zero padding) with ReLU after the first three, on BF16 MFMA with FP32
 * accumulation; parameters and Adam moments FP32.  Volumes are channel-last
 * FP32: inputs [nz][ny][nx][4] = (re x / s_x, im x / s_x, re d / s_d,
 * im d / s_d), outputs and targets [nz][ny][nx][2] = Delta / s_o.  Calls run
 * on the network's stream; buffers grow on demand (the only allocations). */
int cs_cnn_create(void* stream, uint64_t seed, cs_cnn** out);
void cs_cnn_destroy(cs_cnn* n);
const char* cs_cnn_last_error(const cs_cnn* n);
/* parameter count; layout per layer: W [27][cin][cout] (tap = (dz 3 + dy) 3 +
 * dx, offsets d - 1) then b [cout] */
long long cs_cnn_num_params(const cs_cnn* n);
/* host copies of the parameters and/or of the last computed gradient */
int cs_cnn_get_params(cs_cnn* n, float* host, float* grad_host);
int cs_cnn_set_params(cs_cnn* n, const float* host);
/* out = CNN(in): in device [V][4], out device [V][2] */
int cs_cnn_forward(cs_cnn* n, const float* in, int nz, int ny, int nx, float* out);
/* mean over voxels of the squared error summed over the 2 channels, and its
 * gradient (kept for cs_cnn_get_params).  Synchronous. */
int cs_cnn_loss_grad(cs_cnn* n, const float* in, const float* target, int nz, int ny, int nx,
                     double* loss);
/* cs_cnn_loss_grad then one Adam step (beta 0.9, 0.999, eps 1e-8) */
int cs_cnn_train_step(cs_cnn* n, const float* in, const float* target, int nz, int ny, int nx,
                      float lr, double* loss);
/* Training pairs from the sketched solver itself: runs T outer iterations of
 * Algorithm 1 (mode CS_RECON_SKETCH parameters) from x_inout and writes, for
 * outer iteration t, the packed input at inputs + t D 4 and the target
 * (x^{t+1} - x^t) / s_o at targets + t D 2 (device FP32).  l1-wavelet on
 * all coils only: CS_EINVAL for another regularizer, for 0 < C0 < C, for
 * init_iters != 0 and for monitor != 0.  Synchronous. */
int cs_cnn_collect(cs_ctx* ctx, const void* y, const cs_recon_params* p, void* x_inout,
                   float* inputs, float* targets);

/* ---- batches of independent slices ----------------------------------------
 * Many independent reconstructions (slices of uneven size, coil count and
 * sketch size, each with its own context) run Algorithm 1 together.  Every
 * outer iteration runs each slice's full-coil gradient and sketched maps,
 * then the K inner FISTA iterations of all slices as one HIP graph that is
 * captured at the first outer iteration (forked onto the slice streams so
 * that slices overlap) and replayed afterwards. */
typedef struct cs_batch cs_batch;

typedef struct {
  double alpha;                 /* step used by the slice */
  long long n_full_applies;     /* full-coil normal applies in the loop */
  long long n_sketch_applies;   /* sketched normal applies in the loop */
  double wall_prep_ms;          /* host wall time of the set-up (all slices) */
  double wall_loop_ms;          /* host wall time of the T outer iterations (all slices) */
  long long graph_nodes;        /* nodes of the inner-iteration graph (0: eager) */
  long long graph_replays;      /* graph launches */
} cs_batch_stats;

/* Group n contexts (host array ctxs, borrowed; each with its operator set)
 * for batched runs on `stream` (a hipStream_t), which must differ from every
 * slice's own stream; NULL makes the batch create (and destroy) a stream of
 * its own.  Slices may share streams among themselves.  Errors: CS_EINVAL
 * for a null context or a slice on the batch stream, CS_EHIP. */
int cs_batch_create(cs_ctx* const* ctxs, int n, void* stream, cs_batch** out);
void cs_batch_destroy(cs_batch* b);
const char* cs_batch_last_error(const cs_batch* b);

/* Algorithm 1 on every slice: y[i] device [N_i][C_i] (host array of device
 * pointers), p[i] host params (mode CS_RECON_SKETCH, one T and K for all;
 * lam, V, S, seed, t0, step, n_pow per slice; x_ref and reuse_b ignored;
 * l1-wavelet on all coils: CS_EINVAL for another regularizer, for
 * 0 < C0 < C_i, for init_iters != 0 and for monitor != 0), x[i] device [D_i]
 * in/out.  use_graph = 0 issues the inner iterations
 * eagerly (the reference for the graph path: same kernels, same results).
 * st: host array of n (may be NULL).  Synchronous: waits for earlier work on
 * the slice streams first and for all of its own work before returning. */
int cs_batch_recon(cs_batch* b, const void* const* y, const cs_recon_params* p,
                   void* const* x, int use_graph, cs_batch_stats* st);

/* ---- spreading work-group shapes and their autotuner --------------------- */
#define CS_SPREAD_NCFG 13
/* Select spreading shape cfg in [0, CS_SPREAD_NCFG) for this context (all
 * shapes give bit-identical results; they differ only in speed).  Shape 0
 * keeps the sample values of the 3D normal operator in vector registers and
 * broadcasts them with v_readlane; shape 8 does the same and reads a run's
 * LDS voxel when the run opens rather than when it is flushed; shapes 9-11
 * also hold every lane's kernel weights for a whole batch of 64 samples in
 * registers (4 waves x 1 coil, 2 x 2, 1 x 4 per group), and shape 12, the
 * default, is 9 with the values broadcast by DPP row broadcasts instead (in
 * 2D and for the adjoint's caller data, shapes 9-12 run the same
 * register-weight loop with DPP broadcasts on LDS-staged values);
 * shape 7 stages the values in LDS (as every shape does for 2D and for the
 * adjoint's caller data); 1-6 vary the waves and coils per work-group.
 * CS_SPREAD_CFG in the environment sets the default of new operators. */
int cs_set_spread_cfg(cs_ctx* ctx, int cfg);
/* Time a normal apply with the given maps (device [D][ncoil]) under every
 * shape (reps applies each, HIP events on the context stream), select the
 * fastest and report it in *best; ms (host [CS_SPREAD_NCFG], may be NULL)
 * receives the per-apply times.  Cartesian contexts return the current
 * shape.  Synchronous. */
int cs_autotune_spread(cs_ctx* ctx, const void* maps, int ncoil, int reps, int* best,
                       double* ms);

/* Interpolation variant for non-Cartesian contexts (cfg in [0,
 * CS_INTERP_NCFG)): 0 gathers every tap of a sample from the grid in global
 * memory; 1, 2 and 3 (the default) copy each work item's halo'd grid tile
 * into LDS first and gather from there, for coil groups of at most 8 (1), 12
 * (2) or 4 (3) coils in 3D; 4 is 3 with the tile's (re, im) pairs
 * interleaved in LDS (one 8-byte read per tap and coil).  All sum the taps in
 * the same order.  The
 * environment variable CS_INTERP_CFG sets the default of new operators. */
#define CS_INTERP_NCFG 5
int cs_set_interp_cfg(cs_ctx* ctx, int cfg);

/* ---- building blocks exposed for testing and benchmarking ---------------- */

/* Periodized db4 wavelet prox  out = Psi^H soft(Psi v, tau)  (Sec. 2.1,
 * regularizer 2).  v, out device [D] (may alias). */
int cs_prox_l1wav(cs_ctx* ctx, const void* v, float tau, void* out);

/* Forward / inverse db4 transform (Mallat layout), out-of-place, device [D]. */
int cs_dwt(cs_ctx* ctx, const void* x, void* coef);
int cs_idwt(cs_ctx* ctx, const void* coef, void* x);

/* Coil mixing out[d][j] = sum_c in[d][c] * M[j][c] on MFMA (split-BF16,
 * FP32 accumulate).  in device [D][cin], out device [D][cout], M host
 * complex128 [cout][cin] row-major. */
int cs_coil_mix(cs_ctx* ctx, const void* in, int cin, const double* M, int cout,
                void* out);

/* Allocation-free coil mixing, for callers that cannot allocate (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same product as cs_coil_mix, out[d][j] = sum_c in[d][c] * M[j][c] with the
 * same split-BF16 MFMA kernel, but with M in DEVICE memory (complex128
 * [cout][cin] row-major, caller-owned) and its bf16 fragments packed on the
 * GPU into a static 96 KiB scratch array of the library (one per GPU, held
 * until the process ends), so the call makes no allocation, no host copy
 * and no host synchronisation: two kernel launches on the context stream.
 * in device [D][cin], out device [D][cout].  Limit: cin and cout in [1, 64]
 * (CS_EINVAL beyond, before any device work).  Every call on a GPU shares
 * that GPU's scratch, which keeps the last call's fragments: calls that
 * overlap on one GPU (different streams or threads) race and must be
 * ordered by the caller. */
int cs_coil_mix_noalloc(cs_ctx* ctx, const void* in, int cin, const void* M, int cout,
                        void* out);

/* FP64 inner product <a, b> = sum conj(a) b of two device complex64 [D]
 * vectors; result host double[2] (re, im).  Synchronous. */
int cs_dot(cs_ctx* ctx, const void* a, const void* b, double* out);

/* Power iteration on the normal operator with the given maps (Sec. 3.3.1):
 * n_iter normalised applies from the normalised all-ones image; returns
 * L = ||N v_n|| in *L.  Synchronous. */
int cs_power_iteration(cs_ctx* ctx, const void* maps, int ncoil, int n_iter,
                       double* L);

/* Grid dimensions of the operator (NUFFT oversampled grid, or the image for
 * Cartesian), slowest first; m[2] = 1 in 2D. */
int cs_grid_shape(const cs_ctx* ctx, int m[3]);

/* Per-kernel timing with HIP events recorded on the context stream around
 * every kernel launch while enabled.  Kernel kinds (index into the arrays):
 * 0 FFT axis pass, 1 interpolation, 2 spreading, 3 sample gather,
 * 4 wavelet axis pass, 5 soft threshold, 6 element-wise vector op,
 * 7 FP64 reduction, 8 covariance, 9 eigensolver, 10 coil mixing,
 * 11 spreading merge (sum of the halo'd partial tiles).
 * cs_profile_read synchronises, writes the summed milliseconds and launch
 * counts per kind (host arrays of length CS_NKERNELS) and resets them. */
#define CS_NKERNELS 12
int cs_profile_enable(cs_ctx* ctx, int on);
int cs_profile_read(cs_ctx* ctx, double* ms, long long* count);

#ifdef __cplusplus
}
#endif

#endif /* COILSKETCH_H */
