/*
 * cofem.h -- C ABI of libcofem.so, the MI355X (gfx950) hot path of covariance-free
 * EM (CoFEM) for sparse Bayesian learning (Lin, Song, Bilgic, Ba, arXiv 2202.12808).
 *
 * Problem (Sec. 2.1, Eq. 1): y = Phi z + noise, z ~ N(0, diag(alpha)^-1), noise
 * precision beta.  One EM iteration (Algorithm 1) is
 *   A = beta Phi^T Phi + diag(alpha)                        (Eq. 5, Eq. 7)
 *   B = [p_1 .. p_K | beta Phi^T y],  p_k Rademacher       (Eq. 7, Sec. 3.1)
 *   X = [x_1 .. x_K | mu] solves A X = B by CG             (Sec. 3.2)
 *   s = (1/K) sum_k p_k (.) x_k                            (Eq. 6)
 *   alpha <- 1 ./ max(mu (.) mu + s, 1/alpha_max)          (Eq. 8; floor: see below)
 *
 * Conventions for every entry point:
 *  - Pointers documented as "device" are HIP device pointers (e.g. torch CUDA
 *    tensors on ROCm); "host" pointers are ordinary host memory.
 *  - All GPU work is enqueued on the stream given to cofem_init (NULL = the
 *    default stream).  A context is not thread-safe; use one per stream.
 *  - Every call returns a cofem_status; on error, out-parameters are left
 *    untouched and cofem_last_error() describes the failure.  No C++ exception
 *    crosses this boundary.  Reaching the CG iteration cap U is not an error:
 *    the paper caps CG by design (Sec. 3.2) and it shows as converged = 0.
 *  - Readings of the paper fixed by this library: A carries beta in every
 *    section (the CG subsection drops it: a typo); CG starts from X = 0 and
 *    stops once the recursively updated residual satisfies
 *    ||R||_F / ||B||_F < cg_tol (joint Frobenius over all K+1 columns, Sec. 3.2)
 *    or after cg_max_iter iterations; probes are redrawn at every EM iteration
 *    t from the counter-based SplitMix64 stream of `seed` (entry (j, k) takes
 *    bit j mod 64 of stream word (t << 48 | k << 32 | j >> 6), counted from 1;
 *    bit 0 -> +1); the M-step denominator is floored at 1/alpha_max.
 */
#ifndef COFEM_H_
#define COFEM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cofem_status {
  COFEM_OK = 0,
  COFEM_ERR_INVALID_ARG = 1,   /* bad sizes, null pointers, beta <= 0, K out of range */
  COFEM_ERR_OUT_OF_MEMORY = 2, /* device allocation failed (nothing leaked) */
  COFEM_ERR_DEVICE = 3,        /* a HIP runtime call failed; message has hipGetErrorString */
  COFEM_ERR_NUMERIC = 4,       /* NaN/Inf reached a CG scalar */
  COFEM_ERR_UNSUPPORTED = 5    /* a valid request the library does not implement */
} cofem_status;

/* cofem_problem.kind */
enum { COFEM_DENSE = 0, COFEM_CONV2D_CIRC = 1, COFEM_DCT_MASK = 2 };
/* cofem_problem.phi_dtype */
enum { COFEM_F32 = 0, COFEM_BF16 = 1 };
/* cofem_params.precision:
 *  COFEM_PREC_FP32  probe columns in float32 (float64 reductions), mean column
 *                   in float64;
 *  COFEM_PREC_FP64  every column in float64 (convolution dictionaries only)
 *                   -- for ill-conditioned solves whose float32
 *                   probe iterates drift from a float64 reference;
 *  COFEM_PREC_BF16_IR  mixed-precision form (dense only): each E-step solve
 *                   is an iterative refinement whose inner CG solves use Phi
 *                   rounded once to bfloat16 (matrix cores, float32 sums) and
 *                   whose outer residual B - A X uses the float32 Phi with
 *                   float64 sums; it stops when that true residual ratio is
 *                   below cg_tol (the cap U bounds the inner iterations in
 *                   total).  Not in the paper: a precision form layered on
 *                   the solve of Sec. 3.2. */
enum { COFEM_PREC_FP32 = 0, COFEM_PREC_BF16_IR = 1, COFEM_PREC_FP64 = 2 };
/* cofem_params.stop_rule (the stop test of the CG solve, Sec. 3.2):
 *  COFEM_STOP_FROBENIUS   the paper's joint test ||R||_F / ||B||_F < cg_tol on
 *                         the recursively updated residual; every column runs
 *                         the same number of iterations;
 *  COFEM_STOP_PER_COLUMN  column c is finished once ||r_c|| < cg_tol ||b_c||
 *                         (a zero column at once) and takes no further step
 *                         (x_c, r_c frozen); the solve ends when every column
 *                         is finished or at the cap.  Each column then meets
 *                         its own relative tolerance (the mean column b0 is
 *                         ~40..700 times larger than a probe column, so under
 *                         the joint test the probes end less accurate).  Not
 *                         with COFEM_PREC_BF16_IR. */
enum { COFEM_STOP_FROBENIUS = 0, COFEM_STOP_PER_COLUMN = 1 };

/* cofem_params.flags */
enum {
  /* After each CG solve, form the true residual ||B - A X||_F / ||B||_F with
   * one more operator application over X and float64 sums (reported in
   * cofem_iter_stats.rel_resid_true; costs one CG iteration's operator). */
  COFEM_FLAG_TRUE_RESIDUAL = 1,
  /* Batched form: launch each chunk of CG iterations directly instead of
   * replaying the captured graph (same kernels, same results). */
  COFEM_FLAG_EAGER = 2,
  /* Use the batched form (bfloat16 dictionaries) even for n_problems == 1. */
  COFEM_FLAG_BATCHED = 4,
  /* Convolution and DCT dictionaries, and dense ones under
   * COFEM_PREC_BF16_IR, from the second E-step on: start each solve from
   * X0 = [max(s_prev, 0) (.) p_k | mu_prev], the previous E-step's diagonal
   * estimate and mean (not in the paper: a warm start).  The mixed-precision
   * form starts its refinement there: the first outer residual is B - A X0. */
  COFEM_FLAG_WARM_PREV = 8,
  /* Single problems (not the batched form): diagonal (Jacobi)
   * preconditioner M^-1 = 1 / diag(A) = 1 / (beta ||Phi e_d||^2 + alpha_d),
   * recomputed from alpha at every E-step (conv: ||h||^2 for every d; DCT:
   * the column norms of the masked inverse DCT; dense: the column norms of
   * the caller's Phi, summed in float64 once at cofem_init).  Preconditioned
   * CG; the stop test stays the unpreconditioned one of Sec. 3.2.  Under
   * COFEM_PREC_BF16_IR it preconditions the inner solves of the refinement
   * (the outer residual is unchanged). */
  COFEM_FLAG_JACOBI = 16,
  /* Convolution dictionaries (single problems, H and W powers of two, each at
   * most 4096): while alpha is uniform -- the first E-step after cofem_init
   * or cofem_restart, alpha = 1 -- start the solve from X0 = A^-1 B formed by
   * 2D DFTs.  With alpha = a everywhere, A = beta Phi^T Phi + a I (Eq. 3) is
   * block-circulant and the DFT diagonalises it with eigenvalues
   * beta |h_hat|^2 + a, so X0 is the exact solve up to single-precision
   * rounding (complex float32 transforms); CG's stop test (Sec. 3.2) then
   * judges X0 and corrects it, usually in one to three iterations (not in the
   * paper: a start).  Later E-steps start as the other flags say.  After
   * cofem_set_alpha alpha counts as non-uniform until cofem_restart.  Costs
   * ceil((K + T)/2) * D * 8 bytes of transform workspace plus D * 4 bytes of
   * eigenvalue table. */
  COFEM_FLAG_SPECTRAL_START = 32
};

/* Maximum number of probe vectors K per problem. */
#define COFEM_MAX_K 32

/*
 * One SBL problem (Eq. 1).  Dictionary given either densely or as a 2D
 * circular convolution (a structured Phi with a fast apply, Sec. 1, Sec. 3.2).
 *
 * kind == COFEM_DENSE:
 *   phi     device, N x D, row-major with leading dimension ld_phi >= D
 *           (elements), dtype phi_dtype (COFEM_F32).
 * kind == COFEM_CONV2D_CIRC:
 *   N == D == H * W; pixel j = u * W + v (row-major image);
 *   taps    device, kh x kw float32, row-major; kh == kw, odd, 1..9;
 *   (Phi z)[u, v] = sum_{a,b} taps[a, b] * z[(u - a + ch) mod H, (v - b + cw) mod W],
 *   ch = (kh - 1) / 2, cw = (kw - 1) / 2; Phi^T is the matching correlation.
 * kind == COFEM_DCT_MASK (the structured dictionary of Sec. 4: an inverse DCT
 * followed by an undersampling mask):
 *   D = 2^p with 12 <= p <= 20; 1 <= N <= D;
 *   rows    device, N int32: the observed samples, distinct, in [0, D);
 *   (Phi z)_i = (C^T z)[rows[i]] with C the orthonormal DCT-II matrix,
 *   C[k, n] = c_k cos(pi (2n + 1) k / 2D), c_0 = sqrt(1/D), c_k = sqrt(2/D),
 *   so C^T is the inverse DCT and Phi Phi^T = I_N.  Precision COFEM_PREC_FP32
 *   only.  rows is copied to the host once to check it (COFEM_ERR_INVALID_ARG
 *   when an index repeats or is out of range).
 * y         device, N float32; with n_tasks = T > 1, T observation vectors of
 *           N float32 each, task t at y + t N.
 * n_tasks   0 or 1: one observation vector.  T > 1 (COFEM_DCT_MASK only, K + T
 *           <= 64): multi-task SBL, the extension named in Sec. 5: T tasks share
 *           alpha, the E-step solves A X = [p_1 .. p_K | beta Phi^T y_1 .. y_T]
 *           (a float64 column per task), and the M-step is
 *           alpha_j = 1 / max(mean_t mu_tj^2 + s_j, 1/alpha_max).
 *           cofem_posterior then returns task 0's mean; cofem_get_means all.
 * phi, taps, rows and y are read during cofem_init only (the library keeps its
 * own packed copy of Phi or the mask, and the vector beta Phi^T y); the caller
 * keeps ownership.
 */
typedef struct cofem_problem {
  int32_t kind;
  int64_t N;
  int64_t D;
  const void* phi;
  int64_t ld_phi;
  int32_t phi_dtype;
  int32_t H, W, kh, kw;
  const float* taps;
  const float* y;
  const int32_t* rows;
  int32_t n_tasks;
} cofem_problem;

/*
 * Solver parameters: Algorithm 1's beta and K, and the CG controls of
 * Sec. 3.2 (tolerance eps = cg_tol, iteration cap U = cg_max_iter).
 * alpha_max <= 0 selects 1e10.  poll_interval: CG iterations enqueued between
 * host reads of the device stop flag (<= 0 selects a default); it changes
 * nothing in the result, only host/device traffic.
 */
typedef struct cofem_params {
  double beta;
  int32_t K;
  double cg_tol;
  int32_t cg_max_iter;
  uint64_t seed;
  int32_t precision;
  int32_t stop_rule;
  double alpha_max;
  int32_t flags;
  int32_t poll_interval;
  /* COFEM_PREC_BF16_IR only: relative tolerance of each inner solve (0 selects
   * 0.1, the cheapest setting measured on a 4096 x 16384 problem) and the
   * maximum number of refinement sweeps per E-step (0 selects 20) */
  double ir_inner_tol;
  int32_t ir_max_sweeps;
} cofem_params;

/* Per-EM-iteration statistics returned by cofem_em_step (host struct). */
typedef struct cofem_iter_stats {
  int32_t t;           /* EM iteration index that drew the probes */
  int32_t cg_iters;    /* CG iterations run */
  int32_t converged;   /* 1 if the stop test was met before the cap */
  int32_t n_clamped;   /* coordinates whose M-step denominator hit the floor */
  double rel_resid;    /* recursive ||R||_F / ||B||_F at exit */
  double ms;           /* wall time of this EM iteration (device events) */
  double rel_resid_true; /* ||B - A X||_F / ||B||_F at exit, float64 sums
                            (COFEM_FLAG_TRUE_RESIDUAL or COFEM_PREC_BF16_IR), else -1 */
  int32_t ir_sweeps;     /* refinement sweeps (COFEM_PREC_BF16_IR), else 0 */
  double gamma_change;   /* relative change of the prior variances over this
                            M-step, ||1/alpha_new - 1/alpha_old||_2 / ||1/alpha_new||_2
                            (float64 sums; the EM stop test of cofem_em_run) */
} cofem_iter_stats;

typedef struct cofem_ctx cofem_ctx;

/*
 * Creates a context for `n_problems` problems with alpha = 1 (Algorithm 1,
 * first line) and the next EM iteration t = 1, computes beta Phi^T y, and
 * synchronises `hip_stream` before returning.  *out receives the context.
 *
 * Device memory (the packed dictionary and the CG state; dense: 2 packed
 * float32 copies of Phi plus D x 32 float32 blocks; conv: (K) x D float32
 * blocks) comes from one of two places:
 *  - workspace == NULL (workspace_bytes 0): the library allocates it with
 *    hipMalloc and frees it in cofem_destroy;
 *  - workspace != NULL: device memory of workspace_bytes >= the size
 *    cofem_workspace_size reports for the same problems and params, 256-byte
 *    aligned, owned by the caller (e.g. a torch tensor): the context lays its
 *    buffers out in it, allocates no device memory of its own and must be
 *    destroyed before the workspace is freed.  A smaller workspace is
 *    COFEM_ERR_OUT_OF_MEMORY, a misaligned one COFEM_ERR_INVALID_ARG.  The
 *    results are the same bits as with library-allocated memory.
 * (Host-side, the context still takes a few pinned bytes and HIP events.)
 *
 * Batched form (n_problems > 1, phi_dtype == COFEM_BF16, or
 * COFEM_FLAG_BATCHED): independent
 * dense problems sharing beta, K, cg_tol, U; problem i draws its probes with
 * seed + i.  Each Phi_i is rounded to bfloat16 at init (or given in
 * bfloat16) and that bfloat16 matrix is the problem; CG runs in float32
 * with the float64 mean column, all problems' blocks in the same grouped
 * launches, one captured HIP graph replayed per chunk of CG iterations until
 * every problem has stopped.  An autotuner picks the workgroup budget of the
 * grouped passes at init (cofem_batch_plan).  Needs precision
 * COFEM_PREC_FP32 and no COFEM_FLAG_TRUE_RESIDUAL.
 */
cofem_status cofem_init(const cofem_problem* problems, int32_t n_problems,
                        const cofem_params* params, void* hip_stream, void* workspace,
                        size_t workspace_bytes, cofem_ctx** out);

/*
 * The device memory cofem_init needs for these problems and params, in bytes
 * (*bytes, host), so that a caller can provide it as the workspace.  Validates
 * the arguments as cofem_init does; touches no device and reads no device
 * pointer.
 */
cofem_status cofem_workspace_size(const cofem_problem* problems, int32_t n_problems,
                                  const cofem_params* params, size_t* bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one EM
 * iteration of Algorithm 1 for one problem without a context and without any
 * device or pinned allocation.  The same as cofem_init (library-allocated),
 * cofem_set_alpha(alpha_in), cofem_set_iteration(t), cofem_em_step(1) and
 * cofem_posterior(mu, s, alpha_out) followed by cofem_destroy, with the same
 * kernels and the same bits, but every device buffer (packed dictionary, CG
 * state, reduction partials and counters) laid out in a static array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends.  The layout is rebuilt (and cleared) on every call.
 * problem, params: as cofem_init with n_problems = 1; precision
 * COFEM_PREC_FP32 or COFEM_PREC_FP64, no batched form, no
 * COFEM_FLAG_WARM_PREV (COFEM_ERR_UNSUPPORTED otherwise).  A problem whose
 * layout exceeds the 64 MiB (cofem_workspace_size) is COFEM_ERR_INVALID_ARG.
 * alpha_in: device float32, length D (all > 0); t: the EM iteration whose
 * probes are drawn (0..65535); mu, s, alpha_out: device float32, length D,
 * each nullable (alpha_out may equal alpha_in); stats: host, nullable (its
 * ms is host wall time).  Work is enqueued on hip_stream and synchronised
 * before returning.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.
 */
cofem_status cofem_em_step_static(const cofem_problem* problem, const cofem_params* params, const float* alpha_in,
                                  int32_t t, float* mu, float* s, float* alpha_out, cofem_iter_stats* stats,
                                  void* hip_stream);

/*
 * Runs `n_iters` EM iterations of Algorithm 1 (E-step by CG, diagonal
 * estimate, M-step).  The host waits on the stream during each solve (it
 * reads the CG stop flag) and for each iteration's statistics; on return every
 * iteration's device work has completed.  Except for the batched form, the
 * bfloat16 refinement and warm-started dense solves, each iteration's start
 * (predictor, preconditioner, start block) is enqueued before the host waits
 * for the previous iteration's statistics:
 * the device work and its order are those of n_iters calls of one iteration,
 * and so are the results.  `stats` (host, nullable) receives n_iters entries,
 * or n_iters * n_problems for a batched context (entry it * n_problems + i for
 * problem i).
 */
cofem_status cofem_em_step(cofem_ctx* ctx, int32_t n_iters, cofem_iter_stats* stats);

/*
 * Runs EM iterations of Algorithm 1 as cofem_em_step does, but ends early after
 * the first M-step whose gamma_change (the relative change of 1/alpha, see
 * cofem_iter_stats) falls below em_tol: an EM-level stopping rule (the paper
 * runs a fixed T_em; Sec. 4.2 times CoFEM to a target accuracy instead).  At
 * most max_iters iterations; em_tol <= 0 never stops early.  A batched context
 * stops when every problem's change is below em_tol.  stats (host, nullable)
 * receives up to max_iters entries (times n_problems for a batched context),
 * *n_done (host, nullable) the number of EM iterations run.
 */
cofem_status cofem_em_run(cofem_ctx* ctx, int32_t max_iters, double em_tol, cofem_iter_stats* stats,
                          int32_t* n_done);

/*
 * Copies Algorithm 1's return triple for problem `problem`: mu and s of the
 * last E-step and alpha after the last M-step, each into a device float32
 * buffer of length D (each pointer nullable).  Before any EM iteration mu and
 * s are zero.  Enqueued on the context's stream.
 */
cofem_status cofem_posterior(cofem_ctx* ctx, int32_t problem, float* mu, float* s, float* alpha);

/* Replaces alpha of `problem` (device float32, length D, all > 0): the next
 * E-step uses it.  Used for step-by-step comparison with a reference. */
cofem_status cofem_set_alpha(cofem_ctx* ctx, int32_t problem, const float* alpha);

/* The posterior means of every task after the last E-step: mu device, T x D
 * float64 (task t at mu + t D), natural coefficient order.  T = 1 for a
 * single-task context (then mu is cofem_get_solution's mean column). */
cofem_status cofem_get_means(cofem_ctx* ctx, int32_t problem, double* mu);

/* Sets the EM iteration index t (>= 0, < 65536) whose probes the next E-step
 * draws.  The last E-step then no longer precedes the next one, so the
 * previous mean and diagonal estimate are forgotten: the next solve starts
 * from X = 0 (the warm, learned and mixed-precision warm starts resume from
 * the E-step after it). */
cofem_status cofem_set_iteration(cofem_ctx* ctx, int32_t t);

/* Restarts Algorithm 1 from its first line on the same problem: alpha = 1 for
 * every problem, mu = s = 0, t = 1, and no previous solution (the next solve
 * starts from X = 0, exactly as the first E-step of a new context does).
 * Enqueued on the context's stream.  A failed cofem_em_step forgets the
 * previous solution the same way (its iterates may be non-finite). */
cofem_status cofem_restart(cofem_ctx* ctx);

/* n > 0: every CG solve runs exactly n iterations, ignoring cg_tol (the cap is
 * raised to n); n == 0 restores the stop test.  For step-by-step comparisons.
 * COFEM_ERR_UNSUPPORTED under COFEM_PREC_BF16_IR (use cofem_get_ir_sweeps). */
cofem_status cofem_set_fixed_cg_iters(cofem_ctx* ctx, int32_t n);

/*
 * Test and learned-form support: the solution block X of the last E-step.
 * probes: device float32, D x K column-major (column k at probes + k*D);
 * mean: device float64, length D.  Either pointer nullable.
 */
cofem_status cofem_get_solution(cofem_ctx* ctx, int32_t problem, float* probes, double* mean);

/*
 * COFEM_PREC_BF16_IR only: the inner CG iteration count of each refinement
 * sweep of the last E-step.  Writes min(n, capacity) counts to counts (host)
 * and the number of sweeps n to *n (host).
 */
cofem_status cofem_get_ir_sweeps(cofem_ctx* ctx, int32_t* counts, int32_t capacity, int32_t* n);

/*
 * COFEM_PREC_BF16_IR only: applies the inner operator A~ = beta Phi~^T Phi~ +
 * diag(alpha), Phi~ = Phi rounded to bfloat16 (nearest, ties to even), with
 * the inner kernels; arguments as cofem_apply_A.  For operator tests.
 */
cofem_status cofem_apply_A_lowp(cofem_ctx* ctx, int32_t problem, const float* v_probes,
                                const double* v_mean, float* q_probes, double* q_mean);

/*
 * Applies A = beta Phi^T Phi + diag(alpha) of `problem` with the context's
 * own kernels: q_probes = A v_probes (float32, D x K column-major, device)
 * and q_mean = A v_mean (float64, length D, device).  For operator tests.
 */
cofem_status cofem_apply_A(cofem_ctx* ctx, int32_t problem, const float* v_probes,
                           const double* v_mean, float* q_probes, double* q_mean);

/*
 * Writes the Rademacher probe block of EM iteration t (Sec. 3.1) for `seed`:
 * out is device float32, D x K column-major, entries +-1.  Enqueued on
 * hip_stream (NULL = default) and synchronised.  Needs no context.
 */
cofem_status cofem_probe_signs(uint64_t seed, int32_t t, int32_t K, int64_t D, float* out,
                               void* hip_stream);

/*
 * Measurement support: times the operator kernels of one CG iteration in the
 * launch configuration the solver uses, applied to the current direction
 * block: each kernel is launched once to warm up, then `reps` times back to
 * back between two HIP events on the context's stream (the way the CG loop
 * issues it).  Writes the mean per-launch time in milliseconds, dispatch gaps
 * included, of each kernel to ms_out (host, 3 entries):
 * dense -> {pass 1 (W = Phi P), pass 2 (Q = beta Phi^T W + alpha P), 0};
 * batched -> {grouped pass 1, grouped pass 2 over all problems, 0};
 * conv  -> {fused stencil pass, 0, 0}.  Leaves the solver state unchanged.
 */
cofem_status cofem_time_operator(cofem_ctx* ctx, int32_t reps, float* ms_out);

/*
 * Batched form (cofem_init with n_problems > 1, or a COFEM_BF16 dictionary):
 * the autotuner's choice.  *target_wgs: workgroups per operator pass that the
 * grouped launches were planned for (the fastest of 256, 512, 1024, 2048 in
 * a timed trial at init); candidate_ms[4]: the measured ms of one pass-1 +
 * pass-2 pair for each candidate (0 if not tried); splits1/splits2[i]:
 * reduction splits of problem i in pass 1 / pass 2.  Host pointers, each
 * nullable.  COFEM_ERR_UNSUPPORTED for a single-problem context.
 */
cofem_status cofem_batch_plan(cofem_ctx* ctx, int32_t* target_wgs, float* candidate_ms, int32_t* splits1,
                              int32_t* splits2);

/*
 * Learned form (convolution dictionaries; not in the paper): a small network
 * on the image grid predicts, before each E-step from the second on, a start
 * X0 = [d_hat (.) p_k | mu_hat] for the CG solve, which runs preconditioned
 * by the Jacobi diagonal M^-1 = 1/d.  (d_hat estimates diag(Sigma); used as
 * the preconditioner it needs more CG iterations than the Jacobi diagonal.)
 * The solve's stop rule is unchanged (Sec. 3.2), so the prediction only
 * changes how many iterations are needed.
 *
 * Features (5 channels, float32, channel-major H x W images), with the diagonal
 * d = beta ||h||^2 + alpha of A and d_prev from the previous E-step's alpha:
 * alpha/d; mu_prev / rms(mu_prev); log(clip(s_prev d, 1e-3, 1e3)) / 3;
 * log(d / (beta ||h||^2)) / 10; clip(log(d_prev / d), -10, 10) / 10.
 * aux (3 channels): mu_prev, d, sb = clip(s_prev d, 0.05, 20).  Network: four
 * 3x3 circular convolutions, 5 -> 32 -> 32 -> 32 -> 2 channels, ReLU after
 * the first three.  Prediction: mu_hat = mu_prev (1 + tanh o0),
 * d_hat = exp(clip(o1, -10, 10)) sb / d.
 * Loss against an E-step's (mu_t, s_t) (targets, 2 channels), each term relative
 * to the untrained network's (the previous iterate's), with
 * tgt = log(clip(s_t d, 0.05, 20) / sb) and f = 1e-4:
 * sum (mu_hat - mu_t)^2 / (sum (mu_prev - mu_t)^2 + f sum mu_t^2)
 * + 0.1 sum (o1 - tgt)^2 / (sum tgt^2 + f H W).
 * Parameters (float32): for each layer w (Cout x Cin x 3 x 3), then b (Cout).
 * All device pointers below are float32 images of the net's H x W grid.
 */
typedef struct cofem_net cofem_net;

/* Number of network parameters. */
int64_t cofem_net_num_params(void);

/* Creates a network for H x W images: He-normal weights from `seed`, zero
 * biases, zero last layer (untrained, it predicts mu_prev and the clipped
 * previous diagonal estimate, the non-learned warm start).  Work is enqueued on hip_stream. */
cofem_status cofem_net_create(int32_t H, int32_t W, uint64_t seed, void* hip_stream, cofem_net** out);
void cofem_net_destroy(cofem_net* net);

/* Copies all parameters from / to a host float32 array of `count` entries
 * (count must equal cofem_net_num_params()); setting resets Adam's state. */
cofem_status cofem_net_set_params(cofem_net* net, const float* host_params, int64_t count);
cofem_status cofem_net_get_params(cofem_net* net, float* host_params, int64_t count);

/* out (2 channels) = network(feats (5 channels)) in float32 (the training
 * kernels' forward pass); synchronises. */
cofem_status cofem_net_forward(cofem_net* net, const float* feats, float* out);

/* The same forward pass as the predictor runs it (inference): each 3x3 layer
 * an implicit GEMM on bfloat16 MFMA (v_mfma_f32_32x32x16_bf16), weights and
 * activations rounded to bfloat16 (round to nearest even), float32
 * accumulation and float32 activations in memory.  feats (5 images) in, out
 * (2 images) written; synchronises.  COFEM_ERR_INVALID_ARG for a null
 * pointer. */
cofem_status cofem_net_forward_bf16(cofem_net* net, const float* feats, float* out);

/* Loss and its gradient for one sample (feats 5, aux 3, targets 2 channels);
 * *loss (host, nullable) and host_grad (host, cofem_net_num_params() floats,
 * nullable).  Synchronises. */
cofem_status cofem_net_loss_grad(cofem_net* net, const float* feats, const float* aux, const float* targets,
                                 double* loss, float* host_grad);

/* One Adam step (lr; beta1 0.9, beta2 0.999, eps 1e-8) on one sample's
 * gradient; *loss (host, nullable) receives the loss before the step. */
cofem_status cofem_net_train_step(cofem_net* net, const float* feats, const float* aux, const float* targets,
                                  float lr, double* loss);

/* The features and aux channels of the context's next E-step (from its alpha,
 * previous alpha, last mean and last diagonal estimate), written to device
 * buffers of 5 and 3 images; `net` (same H x W) lends its reduction scratch.  Synchronises. */
cofem_status cofem_features(cofem_ctx* ctx, cofem_net* net, float* feats, float* aux);

/* Attaches `net` as the predictor of a convolution context (NULL detaches):
 * from the second E-step on every solve starts from the network's prediction,
 * preconditioned by the Jacobi diagonal.  The net must outlive the
 * attachment. */
cofem_status cofem_set_predictor(cofem_ctx* ctx, cofem_net* net);

/* Kernel slots of cofem_get_kernel_timing. */
enum {
  COFEM_KT_PASS1 = 0,  /* dense: W = Phi P;  conv: the fused iteration (update + stencil pass) */
  COFEM_KT_PASS2 = 1,  /* dense: Q = beta Phi^T W + alpha P with the CG dots;
                        * conv: a solve's first launch, the stencil pass on its start direction */
  COFEM_KT_UPDATE = 2, /* CG update x, r, p and the new residual norms */
  COFEM_KT_INIT = 3,   /* probes, R = P = B, X = 0 */
  COFEM_KT_MSTEP = 4,  /* diagonal estimate and M-step */
  COFEM_KT_CHECK = 5,  /* true-residual check: operator over X and the residual sums */
  COFEM_KT_SLOTS = 6
};

/*
 * Measurement support inside the solver itself.  enable = n > 0 makes every
 * following cofem_em_step record HIP events on the context's stream: one
 * before each launch of every n-th CG iteration (counted over all solves since
 * this call; n = 1 times them all) and of the set-up, check and M-step
 * launches, and an end marker after the last launch of each timed stretch.
 * The totals are reset; 0 turns the recording off, a negative n is
 * COFEM_ERR_INVALID_ARG.  A launch lasts from its event to the next one, so a
 * duration includes the dispatch gap.  Each event costs about a microsecond
 * of stream time: n = 13 keeps the solver within a few percent of its untimed
 * speed.  Choose n coprime to the polling chunk (8 iterations): the first
 * launch after a host wait starts on an idle queue and runs a few
 * microseconds longer, and a period aligned with the chunks would time only
 * those.  CG launches enqueued after the solve stopped (they return at once)
 * are not counted.
 */
cofem_status cofem_set_kernel_timing(cofem_ctx* ctx, int32_t enable);

/*
 * Totals since the last cofem_set_kernel_timing: ms_total[slot] is the summed
 * duration in milliseconds and launches[slot] the number of launches counted,
 * for the COFEM_KT_* slots (host arrays of COFEM_KT_SLOTS entries each).
 */
cofem_status cofem_get_kernel_timing(cofem_ctx* ctx, double* ms_total, int64_t* launches);

/*
 * The name of the kernel that the COFEM_KT_PASS1 or COFEM_KT_PASS2 timing
 * slot times for this context (its kind, precision and problem shape decide
 * it: the convolution dictionary's fused iteration and operator pass run as
 * k_conv_ws, the persistent warp-specialised form, once every workgroup of
 * one per compute unit gets four or more tiles, else as the per-tile
 * k_conv_fused and k_conv_pass; the
 * environment variable COFEM_CONV_KERNEL=tile|ws|ws:<workgroups>, read by
 * cofem_init, overrides that choice), or NULL for a null context or another
 * slot.  A static string; for measurement and profiling tools.
 */
const char* cofem_kernel_name(const cofem_ctx* ctx, int32_t slot);

/* Frees every device buffer of the context (after synchronising its stream). */
void cofem_destroy(cofem_ctx* ctx);

/* Last error message of `ctx` (or of the last failed context-less call when
 * ctx is NULL); never NULL; valid until the next call on the same context. */
const char* cofem_last_error(const cofem_ctx* ctx);

/* Name of a status code. */
const char* cofem_status_string(cofem_status s);

#ifdef __cplusplus
}
#endif

#endif /* COFEM_H_ */
