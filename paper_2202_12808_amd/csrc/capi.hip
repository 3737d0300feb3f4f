// Host runtime and C ABI of libcofem.so: context set-up, the EM driver of
// Algorithm 1 (arXiv 2202.12808) and the test hooks declared in cofem.h.
//
// Per EM iteration t the driver enqueues: the initial-residual kernel (probes
// drawn from the counter-based generator, R = P = B, X = 0), chunks of CG
// iterations (operator pass(es) then the update kernel), and the fused
// diagonal-estimate + M-step kernel.  Every kernel of a CG iteration first
// reads the device stop flag and returns at once when the solve has finished,
// so the host can enqueue a chunk of iterations and read the flag only at the
// end of each chunk: the result is the same as testing after every iteration.
#include "cofem.h"
#include "cofem_internal.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace cofem;

// Host side of the batched form (n_problems > 1 or a bfloat16 dictionary):
// per-problem descriptors and buffers, the grouped launches' work lists, and
// the captured graph of a chunk of CG iterations.
struct BatchHost {
  int n = 0;
  std::vector<cofem::BatchProblem> probs;  // device pointers, host copy
  std::vector<cofem::DenseDims> dims;
  cofem::BatchProblem* d_probs = nullptr;
  cofem::BatchItem *d_items1 = nullptr, *d_items2 = nullptr, *d_itemsv = nullptr;
  int n1 = 0, n2 = 0, nv = 0;
  int32_t* d_running = nullptr;
  int32_t* h_running = nullptr;    // pinned
  cofem::CgScalars* h_st = nullptr;  // pinned, n entries
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool eager = false;
  int chunk = 8;
  int target = 0;                 // chosen workgroups per pass (autotuner)
  float cand_ms[4] = {0.f, 0.f, 0.f, 0.f};
  static constexpr int kCandidates[4] = {256, 512, 1024, 2048};
  static constexpr int kSmax = 8;
};

struct cofem_ctx {
  int kind = COFEM_DENSE;
  BatchHost* batch = nullptr;
  int64_t N = 0, D = 0;
  int K = 0, KP = 0;
  int NT = 1;  // mean columns: tasks sharing alpha
  double beta = 1.0, tol = 1e-5, alpha_max = 1e10;
  int U = 400;
  uint64_t seed = 0;
  int poll = 8;
  int t_next = 1;
  int fixed_iters = 0;
  int prev_iters = 0;
  int precision = COFEM_PREC_FP32;
  bool per_col = false;  // COFEM_STOP_PER_COLUMN
  bool true_resid = false;
  int flags = 0;
  // mixed-precision form (COFEM_PREC_BF16_IR): inner tolerance, sweep cap,
  // bfloat16 copies of Phi, the accumulated solution and the last sweep counts
  double tol_in = 0.1;
  int max_sweeps = 20;
  uint16_t *phiA16 = nullptr, *phiB16 = nullptr;
  float* Xt = nullptr;
  double* xtm = nullptr;
  std::vector<int32_t> sweeps;
  // warm-started / preconditioned / learned forms (conv): M^-1 and the start
  float* minv = nullptr;
  float* dense_cn = nullptr;  // dense Jacobi: ||Phi e_d||^2 (Dp floats)
  float* d0 = nullptr;
  double* mu0 = nullptr;
  const float* active_minv = nullptr;
  // predictor hook (learned form): fills d0 (probe start scale and M^-1) and
  // mu0 (mean start) for the next E-step from the context's current state
  cofem_status (*predictor)(cofem_ctx*, void*, float*, double*) = nullptr;
  void* predictor_user = nullptr;
  bool has_solution = false;
  // spectral start (COFEM_FLAG_SPECTRAL_START): |h_hat|^2, twiddles, the
  // transform workspace; alpha is known to be uniform (= alpha_a0) from
  // cofem_init / cofem_restart until the first M-step or cofem_set_alpha
  float* spec_g = nullptr;
  float2* spec_tw = nullptr;
  float2* spec_z = nullptr;
  bool alpha_uniform = false;
  double alpha_a0 = 1.0;
  hipStream_t stream = nullptr;
  int device = 0;
  DenseDims dd{};
  ConvDims cd{};
  // DCT dictionary: transform geometry and buffers (the CG state uses the conv
  // fields, in the row order of cd.perm)
  DctDims xd{};
  DctBuffers xb{};
  std::vector<void*> allocs;
  // device memory: a caller's workspace (sub-allocated in order, 256-byte
  // aligned) or, when ws is null, one hipMalloc per buffer (allocs).  With
  // `sizing` set nothing is allocated or launched: alloc only counts bytes.
  char* ws = nullptr;
  size_t ws_size = 0, ws_used = 0;
  bool sizing = false;
  // dictionary
  float* phiA = nullptr;
  float* phiB = nullptr;
  float* taps = nullptr;
  // solve state
  double* b0 = nullptr;
  float* alpha = nullptr;
  float* alpha_prev = nullptr;  // conv: the alpha of the last E-step (learned form's features)
  double* dct_cn = nullptr;     // DCT: ||Phi e_k||^2 (state order), for the Jacobi preconditioner
  float *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr;
  double *xm = nullptr, *rm = nullptr, *pm = nullptr, *qm = nullptr;
  // conv probe blocks (float or double per the precision mode)
  void *vX = nullptr, *vR = nullptr, *vP = nullptr, *vQ = nullptr, *vVs = nullptr, *vQs = nullptr;
  // conv: the second buffer set of p, r, q (fused iterations alternate sets)
  void *vP2 = nullptr, *vR2 = nullptr, *vQ2 = nullptr;
  double *pm2 = nullptr, *rm2 = nullptr, *qm2 = nullptr;
  // scratch for apply_A
  float *Vs = nullptr, *Qs = nullptr;
  double *Vsm = nullptr, *Qsm = nullptr;
  // dense GEMM intermediates
  float* W = nullptr;
  double* wm = nullptr;
  float *Wpart = nullptr, *Qpart = nullptr;  // split-K partials
  double *wmpart = nullptr, *qmpart = nullptr;
  uint32_t *cnt_split1 = nullptr, *cnt_split2 = nullptr;
  // reduction workspaces (tree partials and their self-resetting counters)
  double *parts_init = nullptr, *parts_upd = nullptr, *parts_pass = nullptr;
  uint32_t *cnts_init = nullptr, *cnts_upd = nullptr, *cnts_pass = nullptr;
  ConvReduce red_init{}, red_upd{}, red_pass{};
  CgScalars* st = nullptr;
  CgScalars* host_st = nullptr;  // pinned
  CgScalars* host_end = nullptr; // pinned (host_st + 1): the state after an EM iteration's M-step
  // outputs of the last E-step / M-step
  float *mu = nullptr, *sdiag = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_state = nullptr;  // completion of the state copy of a poll
  hipEvent_t ev_end = nullptr;    // completion of the copy into host_end
  hipEvent_t ev0_alt = nullptr;   // the next EM iteration's start while one is finished
  double t0_host = 0.0;           // host clock at the start of an EM iteration
  // optional per-kernel timing: one event before each timed launch, an end
  // marker after the last; CG iterations timed every kt_every-th
  bool ktime = false;
  int kt_every = 1;
  int64_t kt_seq = 0;
  std::vector<hipEvent_t> kev;
  std::vector<int> kev_slot, kev_iter;  // kernel slot and CG iteration of launch i
  size_t kev_used = 0;
  double kt_ms[COFEM_KT_SLOTS] = {};
  int64_t kt_n[COFEM_KT_SLOTS] = {};
  int cg_enq = 0;  // CG iterations enqueued in the current solve
  std::string err;
};

namespace {

thread_local std::string g_err;

cofem_status predictor_hook(cofem_ctx* c, void* user, float* d0, double* mu0);

cofem_status fail(cofem_ctx* c, cofem_status s, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return s;
}

#define COFEM_HIP(ctx, call)                                                                  \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((ctx), e_ == hipErrorOutOfMemory ? COFEM_ERR_OUT_OF_MEMORY : COFEM_ERR_DEVICE, \
                  std::string(#call) + ": " + hipGetErrorString(e_));                         \
  } while (0)

constexpr size_t kWsAlign = 256;

template <typename T>
cofem_status alloc(cofem_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  const size_t bytes = (count == 0 ? 1 : count) * sizeof(T);
  const size_t span = (bytes + kWsAlign - 1) / kWsAlign * kWsAlign;
  if (c->sizing) {
    // counting pass of cofem_workspace_size: a placeholder that is never used
    c->ws_used += span;
    *p = reinterpret_cast<T*>(kWsAlign);
    return COFEM_OK;
  }
  hipError_t e = hipSuccess;
  if (c->ws) {
    if (c->ws_used + span > c->ws_size)
      return fail(c, COFEM_ERR_OUT_OF_MEMORY,
                  "workspace of " + std::to_string(c->ws_size) + " bytes is too small (cofem_workspace_size)");
    q = c->ws + c->ws_used;
    c->ws_used += span;
  } else {
    e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, e == hipErrorOutOfMemory ? COFEM_ERR_OUT_OF_MEMORY : COFEM_ERR_DEVICE,
                  "hipMalloc of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    }
    c->allocs.push_back(q);
  }
  *p = static_cast<T*>(q);
  e = hipMemsetAsync(q, 0, bytes, c->stream);
  if (e != hipSuccess) return fail(c, COFEM_ERR_DEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  return COFEM_OK;
}

#define COFEM_TRY(expr)              \
  do {                               \
    cofem_status s_ = (expr);        \
    if (s_ != COFEM_OK) return s_;   \
  } while (0)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Per-EM-iteration timing: device events when the context has them, else the
// host clock around the iteration (the allocation-free entry point creates
// no events; it synchronises before reading the clock anyway).
double host_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
cofem_status iter_start(cofem_ctx* c) {
  c->t0_host = host_ms();
  if (c->ev0) COFEM_HIP(c, hipEventRecord(c->ev0, c->stream));
  return COFEM_OK;
}
cofem_status iter_end(cofem_ctx* c) {
  if (c->ev1) COFEM_HIP(c, hipEventRecord(c->ev1, c->stream));
  return COFEM_OK;
}
// After the stream has been synchronised past iter_end.
cofem_status iter_ms(cofem_ctx* c, float* ms) {
  if (c->ev0 && c->ev1) {
    COFEM_HIP(c, hipEventElapsedTime(ms, c->ev0, c->ev1));
  } else {
    *ms = (float)(host_ms() - c->t0_host);
  }
  return COFEM_OK;
}

void destroy_ctx(cofem_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->host_st) (void)hipHostFree(c->host_st);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev_state) (void)hipEventDestroy(c->ev_state);
  if (c->ev_end) (void)hipEventDestroy(c->ev_end);
  if (c->ev0_alt) (void)hipEventDestroy(c->ev0_alt);
  for (hipEvent_t e : c->kev) (void)hipEventDestroy(e);
  if (BatchHost* b = c->batch) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->h_running) (void)hipHostFree(b->h_running);
    if (b->h_st) (void)hipHostFree(b->h_st);
    delete b;
  }
  delete c;
}

// Writes the solver controls (cap, tolerance, sizes) into the device scalars.
cofem_status push_controls(cofem_ctx* c) {
  const int n = c->batch ? c->batch->n : 1;
  CgScalars h;
  memset(&h, 0, sizeof(h));
  h.tol = c->precision == COFEM_PREC_BF16_IR ? c->tol_in : c->tol;
  h.limit = c->fixed_iters > 0 ? c->fixed_iters : c->U;
  h.fixed = c->fixed_iters > 0 ? 1 : 0;
  h.kp = c->KP;
  h.k = c->K;
  h.nt = c->NT;
  h.per_col = c->per_col ? 1 : 0;
  h.stop = 1;
  for (int i = 0; i < n; ++i)
    COFEM_HIP(c, hipMemcpyAsync(c->st + i, &h, sizeof(h), hipMemcpyHostToDevice, c->stream));
  COFEM_HIP(c, hipStreamSynchronize(c->stream));
  return COFEM_OK;
}

// Tree-reduction workspace for a grid of nblk blocks with ncols values each.
cofem_status alloc_tree(cofem_ctx* c, double** parts, uint32_t** cnts, int64_t nblk, int ncols,
                        int regions = 1) {
  COFEM_TRY(alloc(c, parts, (size_t)(tree_rows(nblk) * ncols * regions)));
  COFEM_TRY(alloc(c, cnts, (size_t)(tree_counters(nblk) * regions * kCounterStride)));
  return COFEM_OK;
}

cofem_status init_dense(cofem_ctx* c, const cofem_problem& p) {
  DenseDims& dd = c->dd;
  dd.N = p.N;
  dd.D = p.D;
  dd.Np = round_up(p.N, 64);
  dd.Dp = round_up(p.D, 64);
  dd.nt = c->NT;
  dd.S1 = dense_split(dd.Np / 32, dd.Dp / 8, dd.nt);
  dd.S2 = dense_split(dd.Dp / 32, dd.Np / 8, dd.nt);
  dd.ring = 4;
  // tuning override: COFEM_GEMM="S1,S2,ring"
  if (const char* e = getenv("COFEM_GEMM")) {
    int s1, s2, rg;
    if (sscanf(e, "%d,%d,%d", &s1, &s2, &rg) == 3 && dense_split_ok(dd.Dp / 8, s1, dd.nt) &&
        dense_split_ok(dd.Np / 8, s2, dd.nt) && s1 <= 64 && s2 <= 64 &&
        (rg == 1 || rg == 2 || rg == 4 || rg == 8)) {
      dd.S1 = s1;
      dd.S2 = s2;
      dd.ring = rg;
    }
  }
  dd.S1h = dense16_split(dd.Np / 64, dd.Dp / 16);
  dd.S2h = dense16_split(dd.Dp / 64, dd.Np / 16);
  c->KP = kDenseKP;
  const bool lowp = c->precision == COFEM_PREC_BF16_IR;
  const int s1 = lowp && dd.S1h > dd.S1 ? dd.S1h : dd.S1;
  const int s2 = lowp && dd.S2h > dd.S2 ? dd.S2h : dd.S2;

  const size_t blk = (size_t)dd.Dp * kDenseKP, DT = (size_t)dd.Dp * dd.nt;
  COFEM_TRY(alloc(c, &c->phiA, (size_t)dd.Np * dd.Dp));
  COFEM_TRY(alloc(c, &c->phiB, (size_t)dd.Np * dd.Dp));
  COFEM_TRY(alloc(c, &c->b0, DT));  // one float64 column per task
  COFEM_TRY(alloc(c, &c->alpha, dd.Dp));
  COFEM_TRY(alloc(c, &c->mu, dd.Dp));
  COFEM_TRY(alloc(c, &c->sdiag, dd.Dp));
  COFEM_TRY(alloc(c, &c->X, blk));
  COFEM_TRY(alloc(c, &c->R, blk));
  COFEM_TRY(alloc(c, &c->P, blk));
  COFEM_TRY(alloc(c, &c->Q, blk));
  COFEM_TRY(alloc(c, &c->Vs, blk));
  COFEM_TRY(alloc(c, &c->Qs, blk));
  double** vecs[6] = {&c->xm, &c->rm, &c->pm, &c->qm, &c->Vsm, &c->Qsm};
  for (double** v : vecs) COFEM_TRY(alloc(c, v, DT));
  COFEM_TRY(alloc(c, &c->W, (size_t)dd.Np * kDenseKP));
  COFEM_TRY(alloc(c, &c->wm, (size_t)dd.Np * dd.nt));
  const int64_t nupd = dense_update_blocks(dd);
  const int ncols = kDenseKP + dd.nt;
  const bool jacobi = (c->flags & COFEM_FLAG_JACOBI) != 0;
  // the preconditioned start reduces three values per column, its update two
  COFEM_TRY(alloc_tree(c, &c->parts_init, &c->cnts_init, nupd, jacobi ? 3 * ncols : ncols));
  COFEM_TRY(alloc_tree(c, &c->parts_upd, &c->cnts_upd, nupd, jacobi ? 2 * ncols : ncols));
  if (jacobi) {
    COFEM_TRY(alloc(c, &c->dense_cn, dd.Dp));
    COFEM_TRY(alloc(c, &c->minv, dd.Dp));
  }
  COFEM_TRY(alloc_tree(c, &c->parts_pass, &c->cnts_pass, dd.Dp / 32, 3 * ncols));
  COFEM_TRY(alloc(c, &c->Wpart, (size_t)(s1 > 1 ? s1 : 0) * dd.Np * kDenseKP));
  COFEM_TRY(alloc(c, &c->wmpart, (size_t)(s1 > 1 ? s1 : 0) * dd.Np * dd.nt));
  COFEM_TRY(alloc(c, &c->Qpart, (size_t)(s2 > 1 ? s2 : 0) * dd.Dp * kDenseKP));
  COFEM_TRY(alloc(c, &c->qmpart, (size_t)(s2 > 1 ? s2 : 0) * dd.Dp * dd.nt));
  if (lowp) {
    COFEM_TRY(alloc(c, &c->phiA16, (size_t)dd.Np * dd.Dp));
    COFEM_TRY(alloc(c, &c->phiB16, (size_t)dd.Np * dd.Dp));
  }
  if (lowp || (c->flags & COFEM_FLAG_WARM_PREV)) {
    COFEM_TRY(alloc(c, &c->Xt, blk));
    COFEM_TRY(alloc(c, &c->xtm, dd.Dp));
  }
  COFEM_TRY(alloc(c, &c->cnt_split1, (size_t)(dd.Np / 32 * kCounterStride)));
  COFEM_TRY(alloc(c, &c->cnt_split2, (size_t)(dd.Dp / 32 * kCounterStride)));
  if (c->sizing) return COFEM_OK;

  COFEM_HIP(c, dense_pack(static_cast<const float*>(p.phi), p.ld_phi, dd, c->phiA, c->phiB, c->stream));
  if (lowp)
    COFEM_HIP(c, dense_pack16(p.phi, kDictF32ToBf16, p.ld_phi, dd, c->phiA16, c->phiB16, c->stream));
  for (int t = 0; t < dd.nt; ++t)
    COFEM_HIP(c, dense_b0(p.phi, kDictF32, p.ld_phi, p.y + (size_t)t * p.N, c->beta, dd, c->b0 + (size_t)t * dd.Dp,
                          c->stream));
  if (jacobi) COFEM_HIP(c, dense_colnorms(p.phi, kDictF32, p.ld_phi, dd, c->dense_cn, c->stream));
  COFEM_HIP(c, fill_f32(c->alpha, 1.0f, dd.Dp, c->stream));
  return COFEM_OK;
}

// Dense Jacobi diagonal of this E-step's A (COFEM_FLAG_JACOBI), else none.
cofem_status dense_set_minv(cofem_ctx* c) {
  c->active_minv = nullptr;
  if (!c->dense_cn) return COFEM_OK;
  COFEM_HIP(c, dense_jacobi(c->dd, c->dense_cn, c->beta, c->alpha, c->minv, c->stream));
  c->active_minv = c->minv;
  return COFEM_OK;
}

cofem_status init_conv(cofem_ctx* c, const cofem_problem& p) {
  ConvDims& cd = c->cd;
  cd.H = p.H;
  cd.W = p.W;
  cd.ks = p.kh;
  cd.D = (int64_t)p.H * p.W;
  cd.ldD = round_up(cd.D, 256);
  cd.K = c->K;
  cd.tilesX = (p.W + kConvTile - 1) / kConvTile;
  cd.tilesY = (p.H + kConvTile - 1) / kConvTile;
  c->KP = c->K;
  cd.fp64 = c->precision == COFEM_PREC_FP64 ? 1 : 0;
  cd.nt = c->NT;
  // the fused CG iteration as one persistent warp-specialised launch (one
  // workgroup per compute unit) once every workgroup gets several tiles;
  // tuning override: COFEM_CONV_KERNEL=tile | ws | ws:<workgroups>
  cd.ws_grid = 0;
  if (!c->sizing && conv_ws_ok(cd)) {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) {
      const int64_t units = (4 * (int64_t)cd.nt + cd.K) * cd.tilesX * cd.tilesY;
      int mode = 0, grid = ncu;
      if (const char* e = getenv("COFEM_CONV_KERNEL")) {
        if (strcmp(e, "tile") == 0) mode = -1;
        else if (strncmp(e, "ws", 2) == 0) {
          mode = 1;
          if (e[2] == ':' && atoi(e + 3) > 0) grid = atoi(e + 3);
        }
      }
      if (mode > 0 || (mode == 0 && units >= 4 * (int64_t)ncu)) cd.ws_grid = (int)(units < grid ? units : grid);
    }
  }
  const size_t blk = (size_t)cd.ldD * c->K, DT = (size_t)cd.ldD * c->NT;
  COFEM_TRY(alloc(c, &c->taps, (size_t)p.kh * p.kw));
  COFEM_TRY(alloc(c, &c->b0, DT));  // one column per task
  COFEM_TRY(alloc(c, &c->alpha, cd.ldD));
  COFEM_TRY(alloc(c, &c->alpha_prev, cd.ldD));
  COFEM_TRY(alloc(c, &c->mu, cd.ldD));
  COFEM_TRY(alloc(c, &c->sdiag, cd.ldD));
  COFEM_TRY(alloc(c, &c->minv, cd.ldD));
  COFEM_TRY(alloc(c, &c->d0, cd.ldD));
  COFEM_TRY(alloc(c, &c->mu0, cd.ldD));
  void** blocks[9] = {&c->vX, &c->vR, &c->vP, &c->vQ, &c->vVs, &c->vQs, &c->vP2, &c->vR2, &c->vQ2};
  for (void** b : blocks) {
    if (cd.fp64) {
      double* q = nullptr;
      COFEM_TRY(alloc(c, &q, blk));
      *b = q;
    } else {
      float* q = nullptr;
      COFEM_TRY(alloc(c, &q, blk));
      *b = q;
    }
  }
  double** vecs[9] = {&c->xm, &c->rm, &c->pm, &c->qm, &c->rm2, &c->pm2, &c->qm2, &c->Vsm, &c->Qsm};
  for (double** v : vecs) COFEM_TRY(alloc(c, v, DT));  // one float64 column per task
  const int ncols = c->K + c->NT;
  const int64_t nupd = conv_update_blocks(cd), npass = conv_pass_blocks(cd);
  ConvReduce* reds[3] = {&c->red_init, &c->red_upd, &c->red_pass};
  // red_pass also serves the start of a preconditioned solve (nupd blocks)
  const int64_t nblks[3] = {nupd, nupd, npass > nupd ? npass : nupd};
  const int nvs[3] = {1, 3, 5};  // the preconditioned start reduces three values, a fused iteration five
  for (int i = 0; i < 3; ++i) {
    COFEM_TRY(alloc_tree(c, &reds[i]->parts, &reds[i]->cnts, nblks[i], nvs[i], ncols));
    COFEM_TRY(alloc(c, &reds[i]->colsum, (size_t)ncols * nvs[i]));
    COFEM_TRY(alloc(c, &reds[i]->cnt_cols, 1));
  }
  const bool spectral = (c->flags & COFEM_FLAG_SPECTRAL_START) != 0;
  if (spectral) {
    COFEM_TRY(alloc(c, &c->spec_g, (size_t)cd.D));
    COFEM_TRY(alloc(c, &c->spec_tw, (size_t)conv_spectral_twiddles(cd)));
    COFEM_TRY(alloc(c, &c->spec_z, (size_t)(conv_spectral_pairs(cd) * cd.D)));
  }
  if (c->sizing) return COFEM_OK;
  COFEM_HIP(c, hipMemcpyAsync(c->taps, p.taps, sizeof(float) * p.kh * p.kw, hipMemcpyDeviceToDevice,
                              c->stream));
  for (int t = 0; t < c->NT; ++t)
    COFEM_HIP(c, conv_b0(cd, c->taps, p.y + (size_t)t * cd.D, c->beta, c->b0 + (size_t)t * cd.ldD, c->stream));
  COFEM_HIP(c, fill_f32(c->alpha, 1.0f, cd.ldD, c->stream));
  COFEM_HIP(c, fill_f32(c->alpha_prev, 1.0f, cd.ldD, c->stream));
  c->alpha_uniform = true;
  c->alpha_a0 = 1.0;
  if (spectral) COFEM_HIP(c, conv_spectral_tables(cd, c->taps, c->spec_g, c->spec_tw, c->stream));
  return COFEM_OK;
}

cofem_status init_dct(cofem_ctx* c, const cofem_problem& p) {
  int l = 0;
  while ((int64_t(1) << l) < p.D) ++l;
  DctDims& xd = c->xd;
  xd.D = p.D;
  xd.l1 = (l + 1) / 2;
  xd.l2 = l / 2;
  xd.K = c->K;
  xd.npairs = (c->K + 1) / 2;
  xd.units = (1 << xd.l1) / 2 + 1;
  xd.nt = c->NT;
  xd.ntd = (c->NT + 1) / 2;
  ConvDims& cd = c->cd;
  cd.H = 1;
  cd.W = (int)p.D;
  cd.ks = 1;
  cd.D = p.D;
  cd.ldD = p.D;
  cd.K = c->K;
  cd.fp64 = 0;
  cd.perm = xd.l1 | (xd.l2 << 8);
  cd.nt = c->NT;
  cd.ws_grid = 0;
  c->KP = c->K;
  // the observed samples must be distinct and in range (checked once, here)
  if (!c->sizing) {
    std::vector<int32_t> hr((size_t)p.N);
    COFEM_HIP(c, hipMemcpyAsync(hr.data(), p.rows, sizeof(int32_t) * (size_t)p.N, hipMemcpyDeviceToHost, c->stream));
    COFEM_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<uint8_t> seen((size_t)p.D, 0);
    for (int32_t r : hr) {
      if (r < 0 || r >= p.D) return fail(c, COFEM_ERR_INVALID_ARG, "rows holds an index outside [0, D)");
      if (seen[(size_t)r]) return fail(c, COFEM_ERR_INVALID_ARG, "rows holds a repeated index");
      seen[(size_t)r] = 1;
    }
  }
  const size_t D = (size_t)p.D, blk = D * (size_t)c->K, DT = D * (size_t)c->NT;
  const int N1 = 1 << xd.l1, N2 = 1 << xd.l2;
  COFEM_TRY(alloc(c, &c->b0, DT));
  COFEM_TRY(alloc(c, &c->alpha, D));
  COFEM_TRY(alloc(c, &c->mu, D));
  COFEM_TRY(alloc(c, &c->sdiag, D));
  void** blocks[6] = {&c->vX, &c->vR, &c->vP, &c->vQ, &c->vVs, &c->vQs};
  for (void** b : blocks) {
    float* q = nullptr;
    COFEM_TRY(alloc(c, &q, blk));
    *b = q;
  }
  double** vecs[6] = {&c->xm, &c->rm, &c->pm, &c->qm, &c->Vsm, &c->Qsm};
  for (double** v : vecs) COFEM_TRY(alloc(c, v, DT));  // one column per task
  float *Wf = nullptr, *tw1f = nullptr, *tw2f = nullptr;
  double *Wd = nullptr, *vb = nullptr, *tw1d = nullptr, *tw2d = nullptr, *rr = nullptr;
  uint8_t* mk = nullptr;
  COFEM_TRY(alloc(c, &Wf, 2 * D * (size_t)xd.npairs));
  COFEM_TRY(alloc(c, &Wd, 2 * D * (size_t)xd.ntd));
  COFEM_TRY(alloc(c, &mk, D));
  COFEM_TRY(alloc(c, &vb, DT));
  COFEM_TRY(alloc(c, &tw1f, (size_t)2 * N1));
  COFEM_TRY(alloc(c, &tw2f, (size_t)2 * N2));
  COFEM_TRY(alloc(c, &tw1d, (size_t)2 * N1));
  COFEM_TRY(alloc(c, &tw2d, (size_t)2 * N2));
  COFEM_TRY(alloc(c, &rr, (size_t)2 * (c->K + c->NT) * xd.units));
  COFEM_TRY(alloc(c, &c->minv, D));
  COFEM_TRY(alloc(c, &c->dct_cn, D));
  c->xb = DctBuffers{Wf, Wd, mk, c->beta / (double)p.D, tw1f, tw2f, tw1d, tw2d, rr};
  const int ncols = c->K + c->NT;
  ConvReduce* reds[3] = {&c->red_init, &c->red_upd, &c->red_pass};
  const int64_t nupd = conv_update_blocks(cd);
  const int64_t nblks[3] = {nupd, nupd, xd.units};
  // init one value per column; the preconditioned start (and the true
  // residual) up to three per column; an iteration up to five per column
  const int nvs[3] = {1, 3, 5};
  for (int i = 0; i < 3; ++i) {
    // the iteration's tree runs per column slot (a float pair or the mean
    // column) with regions of 2 * nv values
    const int regions = i == 2 ? xd.npairs + xd.ntd : ncols;
    COFEM_TRY(alloc_tree(c, &reds[i]->parts, &reds[i]->cnts, nblks[i], i == 2 ? 2 * nvs[i] : nvs[i], regions));
    COFEM_TRY(alloc(c, &reds[i]->colsum, (size_t)ncols * nvs[i]));
    COFEM_TRY(alloc(c, &reds[i]->cnt_cols, 1));
  }
  if (c->sizing) return COFEM_OK;
  COFEM_HIP(c, dct_setup(xd, p.rows, p.N, p.y, c->beta, mk, vb, tw1f, tw2f, tw1d, tw2d, c->xb, c->b0,
                         (c->flags & COFEM_FLAG_JACOBI) ? c->dct_cn : nullptr, c->stream));
  COFEM_HIP(c, fill_f32(c->alpha, 1.0f, cd.ldD, c->stream));
  return COFEM_OK;
}

// Work lists of the grouped launches for a total of about `target`
// workgroups per pass, shared among the problems in proportion to their
// dictionary size (the splits of each problem within its LDS staging bound).
void batch_plan(BatchHost* b, int target, std::vector<BatchItem>* it1, std::vector<BatchItem>* it2,
                std::vector<BatchItem>* itv) {
  double work = 0.0;
  for (const DenseDims& d : b->dims) work += (double)d.Np * (double)d.Dp;
  auto splits = [&](int64_t pairs, int64_t groups, double share) {
    int64_t s = (int64_t)ceil(target * share / (double)pairs);
    int64_t most = groups / 64;  // at least eight 16-wide groups per wave
    if (most > BatchHost::kSmax) most = BatchHost::kSmax;
    if (s > most) s = most;
    const int64_t least = (groups + 255) / 256;  // LDS staging bound of the mean operand
    if (s < least) s = least;
    return (int)(s < 1 ? 1 : s);
  };
  // largest problems first, so the long work items start early
  std::vector<int> order(b->n);
  for (int i = 0; i < b->n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    return (double)b->dims[x].Np * b->dims[x].Dp > (double)b->dims[y].Np * b->dims[y].Dp;
  });
  it1->clear();
  it2->clear();
  itv->clear();
  for (int i : order) {
    const DenseDims& d = b->dims[i];
    BatchProblem& p = b->probs[i];
    const double share = (double)d.Np * (double)d.Dp / work;
    p.S1 = splits(d.Np / 64, d.Dp / 16, share);
    p.S2 = splits(d.Dp / 64, d.Np / 16, share);
    for (int a = 0; a < p.npairs1; ++a)
      for (int sp = 0; sp < p.S1; ++sp) it1->push_back(BatchItem{i, a, sp, 0});
    for (int a = 0; a < p.npairs2; ++a)
      for (int sp = 0; sp < p.S2; ++sp) it2->push_back(BatchItem{i, a, sp, 0});
    for (int a = 0; a < p.nvec; ++a) itv->push_back(BatchItem{i, a, 0, 0});
  }
}

cofem_status batch_upload(cofem_ctx* c, const std::vector<BatchItem>& it1, const std::vector<BatchItem>& it2,
                          const std::vector<BatchItem>& itv) {
  BatchHost* b = c->batch;
  COFEM_HIP(c, hipMemcpyAsync(b->d_probs, b->probs.data(), sizeof(BatchProblem) * b->n, hipMemcpyHostToDevice,
                              c->stream));
  COFEM_HIP(c, hipMemcpyAsync(b->d_items1, it1.data(), sizeof(BatchItem) * it1.size(), hipMemcpyHostToDevice,
                              c->stream));
  COFEM_HIP(c, hipMemcpyAsync(b->d_items2, it2.data(), sizeof(BatchItem) * it2.size(), hipMemcpyHostToDevice,
                              c->stream));
  COFEM_HIP(c, hipMemcpyAsync(b->d_itemsv, itv.data(), sizeof(BatchItem) * itv.size(), hipMemcpyHostToDevice,
                              c->stream));
  COFEM_HIP(c, hipStreamSynchronize(c->stream));
  b->n1 = (int)it1.size();
  b->n2 = (int)it2.size();
  b->nv = (int)itv.size();
  return COFEM_OK;
}

// One CG iteration of every problem: the two grouped operator passes and the
// grouped update (blocks of stopped problems return at once).
cofem_status batch_cg_iteration(cofem_ctx* c, hipStream_t s) {
  BatchHost* b = c->batch;
  COFEM_HIP(c, batch_pass1(b->d_items1, b->n1, b->d_probs, 0, s));
  COFEM_HIP(c, batch_pass2(b->d_items2, b->n2, b->d_probs, c->beta, 0, s));
  COFEM_HIP(c, batch_update(b->d_itemsv, b->nv, b->d_probs, s));
  return COFEM_OK;
}

cofem_status init_batch(cofem_ctx* c, const cofem_problem* problems, int n) {
  BatchHost* b = new (std::nothrow) BatchHost();
  if (!b) return fail(c, COFEM_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->batch = b;
  b->n = n;
  b->probs.resize(n);
  b->dims.resize(n);
  c->KP = kDenseKP;
  b->eager = (c->flags & COFEM_FLAG_EAGER) != 0;
  if (!c->sizing && (hipHostMalloc(reinterpret_cast<void**>(&b->h_running), sizeof(int32_t)) != hipSuccess ||
                      hipHostMalloc(reinterpret_cast<void**>(&b->h_st), sizeof(CgScalars) * n) != hipSuccess))
    return fail(c, COFEM_ERR_DEVICE, "pinned allocation failed");
  for (int i = 0; i < n; ++i) {
    const cofem_problem& q = problems[i];
    DenseDims& d = b->dims[i];
    d.N = q.N;
    d.D = q.D;
    d.Np = round_up(q.N, 64);
    d.Dp = round_up(q.D, 64);
    d.S1 = d.S2 = 1;
    d.S1h = d.S2h = 1;
    d.ring = 4;
    BatchProblem& p = b->probs[i];
    memset(&p, 0, sizeof(p));
    p.N = d.N;
    p.D = d.D;
    p.Np = d.Np;
    p.Dp = d.Dp;
    p.npairs1 = (int32_t)(d.Np / 64);
    p.npairs2 = (int32_t)(d.Dp / 64);
    p.nvec = dense_update_blocks(d);
    p.seed = c->seed + (uint64_t)i;
    const size_t blk = (size_t)d.Dp * kDenseKP;
    uint16_t *a16 = nullptr, *b16 = nullptr;
    double* b0 = nullptr;
    COFEM_TRY(alloc(c, &a16, (size_t)d.Np * d.Dp));
    COFEM_TRY(alloc(c, &b16, (size_t)d.Np * d.Dp));
    COFEM_TRY(alloc(c, &b0, d.Dp));
    p.phiA16 = a16;
    p.phiB16 = b16;
    p.b0 = b0;
    COFEM_TRY(alloc(c, &p.alpha, d.Dp));
    COFEM_TRY(alloc(c, &p.mu, d.Dp));
    COFEM_TRY(alloc(c, &p.sdiag, d.Dp));
    COFEM_TRY(alloc(c, &p.X, blk));
    COFEM_TRY(alloc(c, &p.R, blk));
    COFEM_TRY(alloc(c, &p.P, blk));
    COFEM_TRY(alloc(c, &p.Q, blk));
    COFEM_TRY(alloc(c, &p.W, (size_t)d.Np * kDenseKP));
    COFEM_TRY(alloc(c, &p.xm, d.Dp));
    COFEM_TRY(alloc(c, &p.rm, d.Dp));
    COFEM_TRY(alloc(c, &p.pm, d.Dp));
    COFEM_TRY(alloc(c, &p.qm, d.Dp));
    COFEM_TRY(alloc(c, &p.wm, d.Np));
    COFEM_TRY(alloc(c, &p.Wpart, (size_t)BatchHost::kSmax * d.Np * kDenseKP));
    COFEM_TRY(alloc(c, &p.wmpart, (size_t)BatchHost::kSmax * d.Np));
    COFEM_TRY(alloc(c, &p.Qpart, (size_t)BatchHost::kSmax * d.Dp * kDenseKP));
    COFEM_TRY(alloc(c, &p.qmpart, (size_t)BatchHost::kSmax * d.Dp));
    COFEM_TRY(alloc(c, &p.cnt_split1, (size_t)(p.npairs1 * kCounterStride)));
    COFEM_TRY(alloc(c, &p.cnt_split2, (size_t)(p.npairs2 * kCounterStride)));
    COFEM_TRY(alloc_tree(c, &p.parts_init, &p.cnts_init, p.nvec, kDenseKP + 1));
    COFEM_TRY(alloc_tree(c, &p.parts_upd, &p.cnts_upd, p.nvec, kDenseKP + 1));
    COFEM_TRY(alloc_tree(c, &p.parts_pass, &p.cnts_pass, p.npairs2, 3 * (kDenseKP + 1)));
    p.st = c->st + i;
    if (c->sizing) continue;
    const int kind = q.phi_dtype == COFEM_BF16 ? kDictBf16 : kDictF32ToBf16;
    COFEM_HIP(c, dense_pack16(q.phi, kind, q.ld_phi, d, a16, b16, c->stream));
    COFEM_HIP(c, dense_b0(q.phi, kind, q.ld_phi, q.y, c->beta, d, b0, c->stream));
    COFEM_HIP(c, fill_f32(p.alpha, 1.0f, d.Dp, c->stream));
  }
  COFEM_TRY(alloc(c, &b->d_probs, (size_t)n));
  COFEM_TRY(alloc(c, &b->d_running, 1));
  // work lists sized for the largest candidate
  std::vector<BatchItem> it1, it2, itv;
  size_t m1 = 0, m2 = 0;
  for (int target : BatchHost::kCandidates) {
    batch_plan(b, target, &it1, &it2, &itv);
    m1 = std::max(m1, it1.size());
    m2 = std::max(m2, it2.size());
  }
  COFEM_TRY(alloc(c, &b->d_items1, m1));
  COFEM_TRY(alloc(c, &b->d_items2, m2));
  COFEM_TRY(alloc(c, &b->d_itemsv, itv.size()));
  if (c->sizing) return COFEM_OK;
  COFEM_HIP(c, hipStreamSynchronize(c->stream));

  // autotuner: time the grouped operator passes (apply only, on the zeroed
  // state) for each candidate workgroup budget; keep the fastest
  int forced = 0;
  if (const char* e = getenv("COFEM_BATCH_TARGET")) forced = atoi(e);
  float best = -1.f;
  for (int k = 0; k < 4; ++k) {
    const int target = BatchHost::kCandidates[k];
    if (forced > 0 && target != forced) continue;
    batch_plan(b, target, &it1, &it2, &itv);
    COFEM_TRY(batch_upload(c, it1, it2, itv));
    for (int w = 0; w < 2; ++w) {
      COFEM_HIP(c, batch_pass1(b->d_items1, b->n1, b->d_probs, 1, c->stream));
      COFEM_HIP(c, batch_pass2(b->d_items2, b->n2, b->d_probs, c->beta, 1, c->stream));
    }
    COFEM_HIP(c, hipEventRecord(c->ev0, c->stream));
    const int reps = 5;
    for (int r = 0; r < reps; ++r) {
      COFEM_HIP(c, batch_pass1(b->d_items1, b->n1, b->d_probs, 1, c->stream));
      COFEM_HIP(c, batch_pass2(b->d_items2, b->n2, b->d_probs, c->beta, 1, c->stream));
    }
    COFEM_HIP(c, hipEventRecord(c->ev1, c->stream));
    COFEM_HIP(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    COFEM_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    b->cand_ms[k] = ms / reps;
    if (best < 0.f || b->cand_ms[k] < best) {
      best = b->cand_ms[k];
      b->target = target;
    }
  }
  if (b->target == 0) b->target = BatchHost::kCandidates[1];
  batch_plan(b, b->target, &it1, &it2, &itv);
  COFEM_TRY(batch_upload(c, it1, it2, itv));

  // graph of one chunk of CG iterations plus the running-problem count
  if (!b->eager) {
    COFEM_HIP(c, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    COFEM_HIP(c, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    cofem_status st = COFEM_OK;
    for (int i = 0; i < b->chunk && st == COFEM_OK; ++i) st = batch_cg_iteration(c, b->cap);
    if (st == COFEM_OK && batch_running(b->d_probs, b->n, b->d_running, b->cap) != hipSuccess)
      st = fail(c, COFEM_ERR_DEVICE, "graph capture: running-count launch failed");
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != COFEM_OK) return st;
    if (e != hipSuccess) return fail(c, COFEM_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    b->graph = g;
    COFEM_HIP(c, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  return COFEM_OK;
}

cofem_status em_iteration_batch(cofem_ctx* c, cofem_iter_stats* out) {
  BatchHost* b = c->batch;
  const int t = c->t_next;
  COFEM_HIP(c, hipEventRecord(c->ev0, c->stream));
  COFEM_HIP(c, batch_init(b->d_itemsv, b->nv, b->d_probs, t, c->K, c->stream));
  const int limit = c->fixed_iters > 0 ? c->fixed_iters : c->U;
  int enqueued = 0;
  for (;;) {
    if (b->exec) {
      COFEM_HIP(c, hipGraphLaunch(b->exec, c->stream));
    } else {
      for (int i = 0; i < b->chunk; ++i) COFEM_TRY(batch_cg_iteration(c, c->stream));
      COFEM_HIP(c, batch_running(b->d_probs, b->n, b->d_running, c->stream));
    }
    enqueued += b->chunk;
    COFEM_HIP(c, hipMemcpyAsync(b->h_running, b->d_running, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    COFEM_HIP(c, hipStreamSynchronize(c->stream));
    if (*b->h_running == 0) break;
    if (enqueued > limit + b->chunk)
      return fail(c, COFEM_ERR_DEVICE, "batched CG did not report completion after the iteration cap");
  }
  COFEM_HIP(c, batch_mstep(b->d_itemsv, b->nv, b->d_probs, t, c->K, c->alpha_max, c->stream));
  COFEM_HIP(c, hipEventRecord(c->ev1, c->stream));
  COFEM_HIP(c, hipMemcpyAsync(b->h_st, c->st, sizeof(CgScalars) * b->n, hipMemcpyDeviceToHost, c->stream));
  COFEM_HIP(c, hipStreamSynchronize(c->stream));
  float ms = 0.0f;
  COFEM_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  for (int i = 0; i < b->n; ++i)
    if (b->h_st[i].numeric_error)
      return fail(c, COFEM_ERR_NUMERIC, "non-finite CG scalar in problem " + std::to_string(i) +
                                            " at EM iteration " + std::to_string(t));
  c->has_solution = true;
  c->t_next = t + 1;
  if (out) {
    for (int i = 0; i < b->n; ++i) {
      const CgScalars& h = b->h_st[i];
      out[i].t = t;
      out[i].cg_iters = h.iter;
      out[i].converged = h.ratio < c->tol ? 1 : 0;
      out[i].n_clamped = h.n_clamped;
      out[i].rel_resid = h.ratio;
      out[i].ms = ms;
      out[i].rel_resid_true = -1.0;
      out[i].ir_sweeps = 0;
      out[i].gamma_change = h.gamma_change;
      if (c->per_col) out[i].converged = h.all_done;
    }
  }
  return COFEM_OK;
}

// Drops what a later E-step could start from (the warm and learned starts
// read the previous E-step's mean and diagonal estimate) and the first
// polling chunk's guess: the next E-step starts from X = 0 as the first
// E-step of a fresh context does.
void forget_solution(cofem_ctx* c) {
  c->has_solution = false;
  c->prev_iters = c->fixed_iters;
}

cofem_status validate(const cofem_problem* p, int32_t n, const cofem_params* q, std::string* why) {
  if (!p || !q) return *why = "null problem or params", COFEM_ERR_INVALID_ARG;
  if (n < 1) return *why = "n_problems must be >= 1", COFEM_ERR_INVALID_ARG;
  if (!(q->beta > 0.0) || !isfinite(q->beta)) return *why = "beta must be positive and finite", COFEM_ERR_INVALID_ARG;
  if (q->K < 1 || q->K > COFEM_MAX_K) return *why = "K must be in [1, 32]", COFEM_ERR_INVALID_ARG;
  if (!(q->cg_tol >= 0.0) || !isfinite(q->cg_tol)) return *why = "cg_tol must be >= 0", COFEM_ERR_INVALID_ARG;
  if (q->cg_max_iter < 0) return *why = "cg_max_iter must be >= 0", COFEM_ERR_INVALID_ARG;
  if (q->precision != COFEM_PREC_FP32 && q->precision != COFEM_PREC_FP64 && q->precision != COFEM_PREC_BF16_IR)
    return *why = "unknown precision mode", COFEM_ERR_INVALID_ARG;
  if (q->precision == COFEM_PREC_BF16_IR) {
    if (p->kind != COFEM_DENSE)
      return *why = "COFEM_PREC_BF16_IR is built for dense dictionaries only", COFEM_ERR_UNSUPPORTED;
    if (!(q->ir_inner_tol >= 0.0) || !(q->ir_inner_tol < 1.0))
      return *why = "ir_inner_tol must be in [0, 1) (0 selects 1e-2)", COFEM_ERR_INVALID_ARG;
    if (q->ir_max_sweeps < 0) return *why = "ir_max_sweeps must be >= 0", COFEM_ERR_INVALID_ARG;
  }
  if (q->precision == COFEM_PREC_FP64 && p->kind != COFEM_CONV2D_CIRC)
    return *why = "COFEM_PREC_FP64 is built for convolution dictionaries only", COFEM_ERR_UNSUPPORTED;
  if (q->stop_rule != COFEM_STOP_FROBENIUS && q->stop_rule != COFEM_STOP_PER_COLUMN)
    return *why = "unknown stop rule", COFEM_ERR_INVALID_ARG;
  if (q->stop_rule == COFEM_STOP_PER_COLUMN && q->precision == COFEM_PREC_BF16_IR)
    return *why = "COFEM_STOP_PER_COLUMN is not built for the refinement of COFEM_PREC_BF16_IR",
           COFEM_ERR_UNSUPPORTED;
  if ((q->flags & COFEM_FLAG_JACOBI) && (n != 1 || (q->flags & COFEM_FLAG_BATCHED) || p->phi_dtype != COFEM_F32))
    return *why = "the Jacobi preconditioner is built for single problems (not the batched form)",
           COFEM_ERR_UNSUPPORTED;
  if ((q->flags & COFEM_FLAG_WARM_PREV) && (n != 1 || (q->flags & COFEM_FLAG_BATCHED) || p->phi_dtype != COFEM_F32))
    return *why = "warm starts are built for single problems (not the batched form)", COFEM_ERR_UNSUPPORTED;
  if ((q->flags & COFEM_FLAG_WARM_PREV) && p->kind == COFEM_DENSE && q->stop_rule == COFEM_STOP_PER_COLUMN)
    return *why = "the dense warm start runs the joint Frobenius stop rule", COFEM_ERR_UNSUPPORTED;
  if ((q->flags & COFEM_FLAG_SPECTRAL_START) &&
      (n != 1 || (q->flags & COFEM_FLAG_BATCHED) || p->kind != COFEM_CONV2D_CIRC))
    return *why = "the spectral start is built for single convolution problems", COFEM_ERR_UNSUPPORTED;
  if ((q->flags & COFEM_FLAG_SPECTRAL_START) && !conv_spectral_ok(p->H, p->W))
    return *why = "the spectral start needs power-of-two H and W, each at most 4096", COFEM_ERR_UNSUPPORTED;
  for (int32_t i = 0; i < n; ++i)
    if (p[i].n_tasks > 1 && (n != 1 || (q->flags & COFEM_FLAG_BATCHED) || p[i].phi_dtype != COFEM_F32))
      return *why = "several tasks (n_tasks > 1) are built for single problems (not the batched form)",
             COFEM_ERR_UNSUPPORTED;
  if (p->n_tasks > 1 && p->kind == COFEM_DENSE &&
      (q->precision != COFEM_PREC_FP32 || (q->flags & COFEM_FLAG_WARM_PREV) || p->n_tasks > kMaxDenseTasks))
    return *why = "several tasks on a dense dictionary: plain float32 CG (precision COFEM_PREC_FP32, no warm "
                  "start), at most 4 tasks",
           COFEM_ERR_UNSUPPORTED;
  if (p->n_tasks < 0 || q->K + (p->n_tasks > 1 ? p->n_tasks : 1) > kMaxCols)
    return *why = "n_tasks must be >= 0 with K + n_tasks <= 64", COFEM_ERR_INVALID_ARG;
  if (n > 1 || p->phi_dtype == COFEM_BF16 || (q->flags & COFEM_FLAG_BATCHED)) {
    // batched form: dense problems whose bfloat16 dictionary is the problem
    if (q->precision != COFEM_PREC_FP32)
      return *why = "the batched form runs plain CG (precision COFEM_PREC_FP32)", COFEM_ERR_UNSUPPORTED;
    if (q->flags & COFEM_FLAG_TRUE_RESIDUAL)
      return *why = "COFEM_FLAG_TRUE_RESIDUAL is not built for the batched form", COFEM_ERR_UNSUPPORTED;
    for (int32_t i = 0; i < n; ++i) {
      const cofem_problem& b = p[i];
      if (b.kind != COFEM_DENSE) return *why = "the batched form takes dense problems", COFEM_ERR_UNSUPPORTED;
      if (b.N < 1 || b.D < 1) return *why = "N and D must be >= 1", COFEM_ERR_INVALID_ARG;
      if (!b.phi || !b.y) return *why = "phi or y is null", COFEM_ERR_INVALID_ARG;
      if (b.ld_phi < b.D) return *why = "ld_phi < D", COFEM_ERR_INVALID_ARG;
      if (b.phi_dtype != COFEM_F32 && b.phi_dtype != COFEM_BF16)
        return *why = "phi_dtype must be COFEM_F32 or COFEM_BF16", COFEM_ERR_INVALID_ARG;
      if (b.N > (int64_t)1 << 24 || b.D > (int64_t)1 << 24) return *why = "N or D too large", COFEM_ERR_INVALID_ARG;
    }
    return COFEM_OK;
  }
  if (!p->y) return *why = "y is null", COFEM_ERR_INVALID_ARG;
  if (p->kind == COFEM_DENSE) {
    if (p->N < 1 || p->D < 1) return *why = "N and D must be >= 1", COFEM_ERR_INVALID_ARG;
    if (!p->phi) return *why = "phi is null", COFEM_ERR_INVALID_ARG;
    if (p->ld_phi < p->D) return *why = "ld_phi < D", COFEM_ERR_INVALID_ARG;
    if (p->phi_dtype != COFEM_F32) return *why = "only float32 Phi is built", COFEM_ERR_UNSUPPORTED;
    if (p->N > (int64_t)1 << 30 || p->D > (int64_t)1 << 30) return *why = "N or D too large", COFEM_ERR_INVALID_ARG;
  } else if (p->kind == COFEM_CONV2D_CIRC) {
    if (p->H < 1 || p->W < 1) return *why = "H and W must be >= 1", COFEM_ERR_INVALID_ARG;
    if (!p->taps) return *why = "taps is null", COFEM_ERR_INVALID_ARG;
    if (p->kh != p->kw) return *why = "only square kernels are built", COFEM_ERR_UNSUPPORTED;
    if (p->kh < 1 || p->kh > 9 || p->kh % 2 == 0) return *why = "kernel side must be odd, 1..9", COFEM_ERR_INVALID_ARG;
    if (p->N != (int64_t)p->H * p->W || p->D != p->N) return *why = "conv needs N == D == H*W", COFEM_ERR_INVALID_ARG;
    if ((int64_t)p->H * p->W > (int64_t)1 << 30) return *why = "image too large", COFEM_ERR_INVALID_ARG;
  } else if (p->kind == COFEM_DCT_MASK) {
    if (p->D < ((int64_t)1 << 12) || p->D > ((int64_t)1 << 20) || (p->D & (p->D - 1)) != 0)
      return *why = "the DCT dictionary needs D = 2^p, 12 <= p <= 20", COFEM_ERR_UNSUPPORTED;
    if (p->N < 1 || p->N > p->D) return *why = "the DCT dictionary needs 1 <= N <= D", COFEM_ERR_INVALID_ARG;
    if (!p->rows) return *why = "rows is null", COFEM_ERR_INVALID_ARG;
    if (q->precision != COFEM_PREC_FP32)
      return *why = "the DCT dictionary runs precision COFEM_PREC_FP32", COFEM_ERR_UNSUPPORTED;
  } else {
    return *why = "unknown dictionary kind", COFEM_ERR_INVALID_ARG;
  }
  return COFEM_OK;
}

// Dictionaries whose CG iterations fold the previous update into the first
// launch: a solve of n updates takes n + 1 iterations' launches.
bool folded_update(const cofem_ctx* c) { return c->kind == COFEM_CONV2D_CIRC || c->kind == COFEM_DCT_MASK; }

// Kernel timing: an event is recorded before every launch (and one after the
// last); launch i lasts from event i to event i + 1, dispatch gap included.
cofem_status mark(cofem_ctx* c, int slot, int iter) {
  if (!c->ktime) return COFEM_OK;
  if (c->kev_used == c->kev.size()) {
    hipEvent_t e;
    // timing only: no system-scope fence (cache writeback) at each record
    COFEM_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    c->kev.push_back(e);
    c->kev_slot.push_back(0);
    c->kev_iter.push_back(0);
  }
  COFEM_HIP(c, hipEventRecord(c->kev[c->kev_used], c->stream));
  c->kev_slot[c->kev_used] = slot;
  c->kev_iter[c->kev_used] = iter;
  ++c->kev_used;
  return COFEM_OK;
}

// Closes the open timing interval with an end marker, so that host waits and
// unsampled launches that follow are not charged to the last timed launch.
cofem_status close_mark(cofem_ctx* c) {
  if (!c->ktime || c->kev_used == 0 || c->kev_slot[c->kev_used - 1] < 0) return COFEM_OK;
  return mark(c, -1, 0);
}

// Whether the next CG iteration is timed: every kt_every-th over the solver's
// lifetime (1: all of them).
bool sampled(cofem_ctx* c) { return c->ktime && (c->kt_seq++ % c->kt_every == 0); }

cofem_status cg_mark(cofem_ctx* c, bool samp, int slot, int iter) { return samp ? mark(c, slot, iter) : COFEM_OK; }

// Adds the recorded launches of a finished EM iteration to the totals.  CG
// launches enqueued after the solve stopped (they return at once) are not
// counted: `iters` is the solve's CG count.
// Reads the first `n_marks` marks (all by default) and drops them; marks
// recorded after them (the next EM iteration's start) move to the front.
cofem_status collect_times(cofem_ctx* c, int iters, size_t n_marks = SIZE_MAX) {
  const size_t n = n_marks < c->kev_used ? n_marks : c->kev_used;
  struct Drop {
    cofem_ctx* c;
    size_t n;
    ~Drop() {
      if (n < c->kev_used) {
        std::rotate(c->kev.begin(), c->kev.begin() + n, c->kev.begin() + c->kev_used);
        std::rotate(c->kev_slot.begin(), c->kev_slot.begin() + n, c->kev_slot.begin() + c->kev_used);
        std::rotate(c->kev_iter.begin(), c->kev_iter.begin() + n, c->kev_iter.begin() + c->kev_used);
      }
      c->kev_used -= n;
    }
  } drop{c, n};
  if (!c->ktime || n < 2) return COFEM_OK;
  COFEM_HIP(c, hipEventSynchronize(c->kev[n - 1]));
  for (size_t i = 0; i + 1 < n; ++i) {
    const int slot = c->kev_slot[i];
    if (slot < 0 || slot >= COFEM_KT_SLOTS) continue;
    if ((slot == COFEM_KT_PASS1 || slot == COFEM_KT_PASS2 || slot == COFEM_KT_UPDATE) && c->kev_iter[i] >= iters)
      continue;
    float ms = 0.f;
    COFEM_HIP(c, hipEventElapsedTime(&ms, c->kev[i], c->kev[i + 1]));
    c->kt_ms[slot] += ms;
    c->kt_n[slot] += 1;
  }
  return COFEM_OK;
}

// Conv solves that start from a block X0 and/or use a diagonal preconditioner:
// COFEM_FLAG_WARM_PREV (X0 = [max(s_prev, 0) (.) p_k | mu_prev]),
// COFEM_FLAG_SPECTRAL_START (X0 = A^-1 B by 2D DFTs while alpha is uniform),
// COFEM_FLAG_JACOBI (M^-1 = 1/diag(A)), or a predictor set by the caller.
bool conv_pcg(const cofem_ctx* c) {
  return (c->kind == COFEM_CONV2D_CIRC || c->kind == COFEM_DCT_MASK) &&
         (c->flags & (COFEM_FLAG_WARM_PREV | COFEM_FLAG_JACOBI | COFEM_FLAG_SPECTRAL_START) || c->predictor);
}

// Q = A X into the scratch blocks (no reduction, no stop check).
cofem_status apply_to_scratch(cofem_ctx* c, void* X, double* xm) {
  if (c->kind == COFEM_DCT_MASK) {
    COFEM_HIP(c, dct_rows_in(c->xd, c->xb, nullptr, nullptr, X, nullptr, nullptr, nullptr, xm, nullptr, nullptr,
                             c->st, 0, 1, c->stream));
    COFEM_HIP(c, dct_mid(c->xd, c->xb, c->st, 1, c->stream));
    COFEM_HIP(c, dct_rows_out(c->xd, c->xb, X, nullptr, c->vQs, xm, nullptr, c->Qsm, c->alpha, nullptr, c->red_pass,
                              c->st, 0, 1, c->stream));
  } else {
    COFEM_HIP(c, conv_pass(c->cd, c->taps, X, xm, c->vR, c->rm, c->alpha, c->beta, c->vQs, c->Qsm, c->red_pass,
                           c->st, 1, c->stream));
  }
  return COFEM_OK;
}

cofem_status pcg_jacobi(cofem_ctx* c) {
  if (c->kind == COFEM_DCT_MASK)
    COFEM_HIP(c, dct_jacobi(c->xd, c->dct_cn, c->beta, c->alpha, c->minv, c->stream));
  else
    COFEM_HIP(c, conv_jacobi(c->cd, c->taps, c->beta, c->alpha, c->minv, c->stream));
  return COFEM_OK;
}

cofem_status conv_start_pcg(cofem_ctx* c, int t) {
  const ConvDims& cd = c->cd;
  const float* d0 = nullptr;
  const double* mu0 = nullptr;
  bool start = false, spectral = false;
  c->active_minv = nullptr;
  if (c->predictor && c->has_solution) {
    // learned: X0 = [d (.) p_k | mu_hat] from the network, M^-1 = Jacobi.
    // (The network's diagonal estimate d tracks diag(Sigma); as a
    // preconditioner it, and blends of it with the Jacobi diagonal, need more
    // iterations than the Jacobi diagonal, most of all right after the first
    // M-step, so it serves only as the probe columns' start.)
    COFEM_TRY(c->predictor(c, c->predictor_user, c->d0, c->mu0));
    COFEM_TRY(pcg_jacobi(c));
    d0 = c->d0;
    mu0 = c->mu0;
    c->active_minv = c->minv;
    start = true;
  } else {
    if (c->flags & COFEM_FLAG_JACOBI) {
      COFEM_TRY(pcg_jacobi(c));
      c->active_minv = c->minv;
    }
    if ((c->flags & COFEM_FLAG_SPECTRAL_START) && c->alpha_uniform && c->kind == COFEM_CONV2D_CIRC) {
      // A = beta Phi^T Phi + a0 I is block-circulant: X0 = A^-1 B by 2D DFTs
      COFEM_HIP(c, conv_spectral_start(cd, c->seed, t, c->b0, c->spec_g, c->spec_tw, c->beta, c->alpha_a0,
                                       c->spec_z, c->vX, c->xm, c->stream));
      spectral = true;
      start = true;
    } else if ((c->flags & COFEM_FLAG_WARM_PREV) && c->has_solution) {
      d0 = c->sdiag;  // clamped at zero by conv_start
      start = true;
    }
  }
  // the start's column reduction (conv_update_blocks blocks, three values per
  // column): conv sizes red_pass for it, the DCT dictionary red_upd
  const ConvReduce& rs = c->kind == COFEM_DCT_MASK ? c->red_upd : c->red_pass;
  if (start) {
    if (!spectral) COFEM_HIP(c, conv_start(cd, c->seed, t, d0, mu0, c->vX, c->xm, c->stream));
    if (c->kind == COFEM_CONV2D_CIRC && cd.ws_grid > 0) {
      // the persistent kernel forms R = B - A X0 and P = M^-1 R with their sums
      // in its epilogue (A X0 is not stored)
      COFEM_HIP(c, conv_init_ws(cd, cd.ws_grid, c->taps, c->seed, t, c->b0, c->active_minv, c->vX, c->xm, c->vR,
                                c->vP, c->rm, c->pm, c->alpha, c->beta, c->red_pass, c->st, c->stream));
    } else {
      COFEM_TRY(apply_to_scratch(c, c->vX, c->xm));
      COFEM_HIP(c, conv_init_pcg(cd, c->seed, t, c->b0, c->active_minv, c->vQs, c->Qsm, c->vX, c->vR, c->vP, c->xm,
                                 c->rm, c->pm, rs, c->st, c->stream));
    }
  } else {
    COFEM_HIP(c, conv_init_pcg(cd, c->seed, t, c->b0, c->active_minv, nullptr, nullptr, c->vX, c->vR, c->vP, c->xm,
                               c->rm, c->pm, rs, c->st, c->stream));
  }
  return COFEM_OK;
}

cofem_status run_cg_iterations(cofem_ctx* c, int n, bool lowp = false) {
  COFEM_TRY(close_mark(c));
  for (int i = 0; i < n; ++i) {
    const int it = c->cg_enq++;
    const bool samp = sampled(c);
    if (c->kind == COFEM_DENSE && lowp) {
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_PASS1, it));
      COFEM_HIP(c, dense16_pass1(c->dd, c->phiA16, c->P, c->pm, c->Wpart, c->wmpart, c->W, c->wm,
                                 c->cnt_split1, c->st, 0, c->stream));
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_PASS2, it));
      COFEM_HIP(c, dense16_pass2(c->dd, c->phiB16, c->W, c->wm, c->P, c->pm, c->R, c->rm, c->alpha, c->beta,
                                 c->Qpart, c->qmpart, c->Q, c->qm, c->parts_pass, c->cnts_pass,
                                 c->cnt_split2, c->st, 0, c->stream, c->active_minv));
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_UPDATE, it));
      COFEM_HIP(c, dense_update(c->dd, c->X, c->R, c->P, c->Q, c->xm, c->rm, c->pm, c->qm, c->parts_upd,
                                c->cnts_upd, c->st, c->stream, c->active_minv));
    } else if (c->kind == COFEM_DENSE) {
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_PASS1, it));
      COFEM_HIP(c, dense_pass1(c->dd, c->phiA, c->P, c->pm, c->Wpart, c->wmpart, c->W, c->wm,
                               c->cnt_split1, c->st, 0, c->stream));
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_PASS2, it));
      COFEM_HIP(c, dense_pass2(c->dd, c->phiB, c->W, c->wm, c->P, c->pm, c->R, c->rm, c->alpha, c->beta,
                               c->Qpart, c->qmpart, c->Q, c->qm, c->parts_pass, c->cnts_pass,
                               c->cnt_split2, c->st, 0, c->stream, c->active_minv));
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_UPDATE, it));
      COFEM_HIP(c, dense_update(c->dd, c->X, c->R, c->P, c->Q, c->xm, c->rm, c->pm, c->qm, c->parts_upd,
                                c->cnts_upd, c->st, c->stream, c->active_minv));
    } else if (c->kind == COFEM_DCT_MASK) {
      // DCT: the first iteration of a solve is the operator on the start
      // direction; each later one folds the previous update into its first
      // launch (state updated in place: no launch reads another row's state)
      const int fused = it > 0 ? 1 : 0;
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_PASS1, it));
      COFEM_HIP(c, dct_rows_in(c->xd, c->xb, c->vX, c->vR, c->vP, c->vQ, c->xm, c->rm, c->pm, c->qm,
                               conv_pcg(c) ? c->active_minv : nullptr, c->st, fused, 0, c->stream));
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_PASS2, it));
      COFEM_HIP(c, dct_mid(c->xd, c->xb, c->st, 0, c->stream));
      COFEM_TRY(cg_mark(c, samp, COFEM_KT_UPDATE, it));
      COFEM_HIP(c, dct_rows_out(c->xd, c->xb, c->vP, c->vR, c->vQ, c->pm, c->rm, c->qm, c->alpha,
                                conv_pcg(c) ? c->active_minv : nullptr, c->red_pass, c->st, fused, 0, c->stream));
    } else {
      // conv: the first launch of a solve is the operator pass on the start
      // direction (set 0); each later one a fused iteration, the previous
      // update applied while staging, reading set (it - 1) % 2 and writing
      // set it % 2 (so a solve needs one launch more than it has updates)
      const float* minv = conv_pcg(c) ? c->active_minv : nullptr;
      const ConvState sets[2] = {{c->vP, c->vR, c->vQ, c->pm, c->rm, c->qm},
                                 {c->vP2, c->vR2, c->vQ2, c->pm2, c->rm2, c->qm2}};
      // (timed apart: the fused iterations in the pass-1 slot, a solve's first
      // pass in the pass-2 slot)
      COFEM_TRY(cg_mark(c, samp, it == 0 ? COFEM_KT_PASS2 : COFEM_KT_PASS1, it));
      if (it == 0)
        COFEM_HIP(c, conv_pass(c->cd, c->taps, c->vP, c->pm, c->vR, c->rm, c->alpha, c->beta, c->vQ, c->qm,
                               c->red_pass, c->st, 0, c->stream, minv));
      else
        COFEM_HIP(c, conv_fused(c->cd, c->taps, sets[(it - 1) & 1], sets[it & 1], c->vX, c->xm, c->alpha, c->beta,
                                minv, c->red_pass, c->st, c->stream));
    }
    // close a sampled iteration unless the next one is sampled too
    if (samp && !(i + 1 < n && c->kt_seq % c->kt_every == 0)) COFEM_TRY(close_mark(c));
  }
  return COFEM_OK;
}

// Final check of a solve: Q = A X with the operator kernels (the same
// launches as a CG iteration, applied to X instead of the direction block),
// then ||b_c - q_c||^2 per column in float64 against B regenerated for EM
// iteration t.  Uses alpha of this E-step, so it runs before the M-step.
cofem_status true_residual(cofem_ctx* c, int t) {
  COFEM_TRY(mark(c, COFEM_KT_CHECK, 0));
  if (c->kind == COFEM_DENSE) {
    COFEM_HIP(c, dense_pass1(c->dd, c->phiA, c->X, c->xm, c->Wpart, c->wmpart, c->W, c->wm, c->cnt_split1,
                             c->st, 1, c->stream));
    COFEM_HIP(c, dense_pass2(c->dd, c->phiB, c->W, c->wm, c->X, c->xm, c->R, c->rm, c->alpha, c->beta,
                             c->Qpart, c->qmpart, c->Qs, c->Qsm, c->parts_pass, c->cnts_pass, c->cnt_split2,
                             c->st, 1, c->stream));
    COFEM_HIP(c, dense_true_resid(c->dd, c->seed, t, c->K, c->b0, c->Qs, c->Qsm, c->parts_upd, c->cnts_upd,
                                  c->st, c->stream));
  } else {
    if (c->kind == COFEM_DCT_MASK) {
      COFEM_HIP(c, dct_rows_in(c->xd, c->xb, nullptr, nullptr, c->vX, nullptr, nullptr, nullptr, c->xm, nullptr,
                               nullptr, c->st, 0, 1, c->stream));
      COFEM_HIP(c, dct_mid(c->xd, c->xb, c->st, 1, c->stream));
      COFEM_HIP(c, dct_rows_out(c->xd, c->xb, c->vX, nullptr, c->vQs, c->xm, nullptr, c->Qsm, c->alpha, nullptr,
                                c->red_pass, c->st, 0, 1, c->stream));
    } else if (c->cd.ws_grid > 0) {
      // the persistent kernel sums ||b - A x||^2 in its epilogue (A X is not stored)
      COFEM_HIP(c, conv_resid_ws(c->cd, c->cd.ws_grid, c->taps, c->seed, t, c->b0, c->vX, c->xm, c->alpha, c->beta,
                                 c->red_pass, c->st, c->stream));
      return COFEM_OK;
    } else {
      COFEM_HIP(c, conv_pass(c->cd, c->taps, c->vX, c->xm, c->vR, c->rm, c->alpha, c->beta, c->vQs, c->Qsm,
                             c->red_pass, c->st, 1, c->stream));
    }
    COFEM_HIP(c, conv_true_resid(c->cd, c->seed, t, c->b0, c->vQs, c->Qsm, c->red_upd, c->st, c->stream));
  }
  return COFEM_OK;
}

cofem_status read_state(cofem_ctx* c) {
  COFEM_HIP(c, hipMemcpyAsync(c->host_st, c->st, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
  COFEM_HIP(c, hipStreamSynchronize(c->stream));
  return COFEM_OK;
}

// A poll of a running solve: copies the state as it stands after the
// iterations enqueued so far, then (if `ahead`) enqueues one more CG iteration
// before waiting for the copy, so the GPU is not idle while the host reads the
// flag.  After a stop that iteration returns at once.  Returns the number of
// iterations it enqueued (0 or 1).
// With `resid_t` >= 0 the launch ahead is instead the true residual of EM
// iteration resid_t in the form that runs only if the solve has stopped (the
// persistent conv kernel): the copy is taken just before it, so it runs
// exactly when the host then reads the stop.
cofem_status poll_state(cofem_ctx* c, bool ahead, bool lowp, int* extra, int resid_t = -1) {
  COFEM_HIP(c, hipMemcpyAsync(c->host_st, c->st, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
  if (c->ev_state) COFEM_HIP(c, hipEventRecord(c->ev_state, c->stream));
  *extra = 0;
  if (resid_t >= 0) {
    COFEM_TRY(close_mark(c));
    COFEM_TRY(mark(c, COFEM_KT_CHECK, 0));
    COFEM_HIP(c, conv_resid_ws(c->cd, c->cd.ws_grid, c->taps, c->seed, resid_t, c->b0, c->vX, c->xm, c->alpha,
                               c->beta, c->red_pass, c->st, c->stream, true));
    COFEM_TRY(mark(c, -1, 0));
  } else if (ahead) {
    COFEM_TRY(run_cg_iterations(c, 1, lowp));
    *extra = 1;
  }
  if (c->ev_state)
    COFEM_HIP(c, hipEventSynchronize(c->ev_state));
  else
    COFEM_HIP(c, hipStreamSynchronize(c->stream));
  return COFEM_OK;
}

// Launch plan of a solve.  The first chunk is the previous solve's launch
// count (CG counts drift slowly across EM iterations), so that the poll after
// it sees the stop when the count is unchanged; a cold solve starts with
// `poll` launches.  `folded` is the launch a solve has beyond its updates.
int first_chunk(const cofem_ctx* c, int folded, int limit) {
  const int chunk = c->prev_iters > 0 ? c->prev_iters + folded : c->poll;
  return chunk < limit ? chunk : limit;
}

// The chunk after the `misses`-th poll that did not see the stop (`extra`:
// the launch that poll enqueued ahead).  A predicted solve that ran past the
// previous count is near its end: chunks of 1, 2, 4, ... launches (the poll's
// own launch ahead included) up to `poll`; a cold one takes `poll` at a time.
// Never past the cap, and never an empty round once the cap is reached (no
// launch ahead then).
int next_chunk(const cofem_ctx* c, bool predicted, int misses, int extra, int enqueued, int limit) {
  int want = c->poll;
  if (predicted && misses <= 16 && (1 << (misses - 1)) < want) want = 1 << (misses - 1);
  int chunk = want - extra;
  if (chunk < 0) chunk = 0;
  if (enqueued + chunk > limit) chunk = limit - enqueued > 0 ? limit - enqueued : 1;
  if (chunk == 0 && enqueued >= limit) chunk = 1;
  return chunk;
}

// Mixed-precision E-step (COFEM_PREC_BF16_IR): iterative refinement.  X = 0,
// R = B; each sweep solves A~ D = R by CG with the bfloat16 Phi to the inner
// tolerance (relative to ||R||_F), adds D to X, and forms the outer residual
// R = B - A X with the float32 Phi and float64 sums; the sweeps stop once
// ||R||_F / ||B||_F < eps, after U inner iterations in total, or after
// max_sweeps sweeps.  The M-step then reads the accumulated X.
constexpr int kIrStall = 3;

cofem_status em_iteration_ir(cofem_ctx* c, cofem_iter_stats* out) {
  const int t = c->t_next;
  const DenseDims& dd = c->dd;
  COFEM_TRY(iter_start(c));
  c->kev_used = 0;
  c->sweeps.clear();
  COFEM_TRY(mark(c, COFEM_KT_INIT, 0));
  COFEM_TRY(dense_set_minv(c));
  COFEM_HIP(c, dense_init(dd, c->seed, t, c->K, c->b0, c->X, c->R, c->P, c->xm, c->rm, c->pm, c->parts_init,
                          c->cnts_init, c->st, c->stream, c->active_minv));
  const bool warm = (c->flags & COFEM_FLAG_WARM_PREV) && c->has_solution;
  if (warm) {
    // X0 = [max(s_prev, 0) (.) p_k | mu_prev] (Xt still holds the previous
    // mean), then the first outer residual R = B - A X0 with the float32 Phi,
    // which also sets up the first inner solve
    COFEM_HIP(c, dense_warm_start(dd, c->seed, t, c->K, c->sdiag, c->Xt, c->stream));
    COFEM_HIP(c, dense_pass1(dd, c->phiA, c->Xt, c->xtm, c->Wpart, c->wmpart, c->W, c->wm, c->cnt_split1, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_pass2(dd, c->phiB, c->W, c->wm, c->Xt, c->xtm, c->R, c->rm, c->alpha, c->beta, c->Qpart,
                             c->qmpart, c->Qs, c->Qsm, c->parts_pass, c->cnts_pass, c->cnt_split2, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_ir_residual(dd, c->seed, t, c->K, c->b0, c->Qs, c->Qsm, c->X, c->R, c->P, c->xm, c->rm, c->pm,
                                   c->parts_upd, c->cnts_upd, c->st, c->U, c->stream, c->active_minv));
  } else {
    COFEM_HIP(c, fill_f32(c->Xt, 0.0f, dd.Dp * kDenseKP, c->stream));
    COFEM_HIP(c, hipMemsetAsync(c->xtm, 0, sizeof(double) * dd.Dp, c->stream));
  }
  COFEM_TRY(read_state(c));
  if (warm && c->host_st->numeric_error)
    return fail(c, COFEM_ERR_NUMERIC, "non-finite warm-start residual at EM iteration " + std::to_string(t));
  double outer = warm ? c->host_st->true_ratio : (c->host_st->nB0 > 0.0 ? 1.0 : 0.0), best = outer;
  int total = 0, stall = 0;
  for (;;) {
    // The true residual of refinement need not fall monotonically.  Stop at the
    // tolerance, at the caps, or after kIrStall sweeps in a row without halving
    // the best ratio so far (its float32 evaluation has reached its floor).
    if (!c->sweeps.empty()) {
      if (outer < 0.5 * best) {
        best = outer;
        stall = 0;
      } else {
        ++stall;
      }
    }
    if (outer < c->tol || total >= c->U || (int)c->sweeps.size() >= c->max_sweeps || stall >= kIrStall) break;
    // inner solve with the bfloat16 dictionary
    c->cg_enq = 0;
    int chunk = c->poll, enqueued = 0;
    const int limit = c->U - total;
    if (chunk > limit) chunk = limit;
    for (;;) {
      if (chunk > 0) COFEM_TRY(run_cg_iterations(c, chunk, true));
      enqueued += chunk;
      int extra = 0;
      COFEM_TRY(poll_state(c, enqueued < limit, true, &extra));
      enqueued += extra;
      if (c->host_st->stop) break;
      if (enqueued > limit + 2) return fail(c, COFEM_ERR_DEVICE, "inner CG did not report completion");
      chunk = c->poll - extra;
      if (enqueued + chunk > limit) chunk = limit - enqueued > 0 ? limit - enqueued : 1;
    }
    if (c->host_st->numeric_error)
      return fail(c, COFEM_ERR_NUMERIC, "non-finite value in an inner CG scalar at EM iteration " + std::to_string(t));
    const int n_in = c->host_st->iter;
    COFEM_TRY(mark(c, -1, 0));
    COFEM_TRY(collect_times(c, n_in));
    total += n_in;
    c->sweeps.push_back(n_in);
    // outer residual with the float32 dictionary
    COFEM_TRY(mark(c, COFEM_KT_CHECK, 0));
    COFEM_HIP(c, dense_ir_accumulate(dd, c->Xt, c->X, c->xtm, c->xm, c->stream));
    COFEM_HIP(c, dense_pass1(dd, c->phiA, c->Xt, c->xtm, c->Wpart, c->wmpart, c->W, c->wm, c->cnt_split1, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_pass2(dd, c->phiB, c->W, c->wm, c->Xt, c->xtm, c->R, c->rm, c->alpha, c->beta, c->Qpart,
                             c->qmpart, c->Qs, c->Qsm, c->parts_pass, c->cnts_pass, c->cnt_split2, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_ir_residual(dd, c->seed, t, c->K, c->b0, c->Qs, c->Qsm, c->X, c->R, c->P, c->xm, c->rm, c->pm,
                                   c->parts_upd, c->cnts_upd, c->st, c->U - total, c->stream, c->active_minv));
    COFEM_TRY(mark(c, -1, 0));
    COFEM_TRY(read_state(c));
    COFEM_TRY(collect_times(c, 0));
    if (c->host_st->numeric_error)
      return fail(c, COFEM_ERR_NUMERIC, "non-finite outer residual at EM iteration " + std::to_string(t));
    outer = c->host_st->true_ratio;
  }
  COFEM_TRY(mark(c, COFEM_KT_MSTEP, 0));
  COFEM_HIP(c, dense_mstep(dd, c->seed, t, c->K, c->Xt, c->xtm, c->alpha, c->alpha_max, c->mu, c->sdiag,
                           c->parts_upd, c->cnts_upd, c->st, c->stream));
  COFEM_TRY(mark(c, -1, 0));
  COFEM_TRY(iter_end(c));
  COFEM_TRY(read_state(c));
  COFEM_TRY(collect_times(c, 0));
  c->has_solution = true;
  c->prev_iters = total;
  c->t_next = t + 1;
  if (out) {
    float ms = 0.0f;
    COFEM_TRY(iter_ms(c, &ms));
    out->t = t;
    out->cg_iters = total;
    out->converged = outer < c->tol ? 1 : 0;
    out->n_clamped = c->host_st->n_clamped;
    out->rel_resid = outer;
    out->ms = ms;
    out->rel_resid_true = outer;
    out->ir_sweeps = (int32_t)c->sweeps.size();
    out->gamma_change = c->host_st->gamma_change;
  }
  return COFEM_OK;
}

// Dense float32 CG from the previous E-step's mean and diagonal estimate
// (COFEM_FLAG_WARM_PREV): X0 = [max(s_prev, 0) (.) p_k | mu_prev] in Xt, R0 =
// B - A X0, and plain CG on A D = R0 from D = 0, whose stop test
// ||R||_F / ||R0||_F < eps ||B||_F / ||R0||_F is the solve's own test
// ||R||_F / ||B||_F < eps (Sec. 3.2); X = X0 + D.  The first E-step (no
// previous solution) starts from zero as plain CG does.
cofem_status em_iteration_dense_warm(cofem_ctx* c, cofem_iter_stats* out) {
  const int t = c->t_next;
  const DenseDims& dd = c->dd;
  COFEM_TRY(iter_start(c));
  c->cg_enq = 0;
  c->kev_used = 0;
  COFEM_TRY(mark(c, COFEM_KT_INIT, 0));
  COFEM_TRY(dense_set_minv(c));
  COFEM_HIP(c, dense_init(dd, c->seed, t, c->K, c->b0, c->X, c->R, c->P, c->xm, c->rm, c->pm, c->parts_init,
                          c->cnts_init, c->st, c->stream, c->active_minv));
  const bool warm = c->has_solution;
  double tol_eff = c->tol;
  if (warm) {
    COFEM_HIP(c, dense_warm_start(dd, c->seed, t, c->K, c->sdiag, c->Xt, c->stream));
    COFEM_HIP(c, dense_pass1(dd, c->phiA, c->Xt, c->xtm, c->Wpart, c->wmpart, c->W, c->wm, c->cnt_split1, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_pass2(dd, c->phiB, c->W, c->wm, c->Xt, c->xtm, c->R, c->rm, c->alpha, c->beta, c->Qpart,
                             c->qmpart, c->Qs, c->Qsm, c->parts_pass, c->cnts_pass, c->cnt_split2, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_ir_residual(dd, c->seed, t, c->K, c->b0, c->Qs, c->Qsm, c->X, c->R, c->P, c->xm, c->rm, c->pm,
                                   c->parts_upd, c->cnts_upd, c->st, c->fixed_iters > 0 ? c->fixed_iters : c->U,
                                   c->stream, c->active_minv));
    COFEM_TRY(read_state(c));
    if (c->host_st->numeric_error)
      return fail(c, COFEM_ERR_NUMERIC, "non-finite warm-start residual at EM iteration " + std::to_string(t));
    const double r0 = c->host_st->true_ratio;  // ||R0||_F / ||B||_F
    tol_eff = r0 > 0.0 ? c->tol / r0 : c->tol;
    if (c->fixed_iters > 0) tol_eff = 0.0;
    COFEM_HIP(c, hipMemcpyAsync(&c->st->tol, &tol_eff, sizeof(double), hipMemcpyHostToDevice, c->stream));
  } else {
    COFEM_HIP(c, fill_f32(c->Xt, 0.0f, dd.Dp * kDenseKP, c->stream));
    COFEM_HIP(c, hipMemsetAsync(c->xtm, 0, sizeof(double) * dd.Dp, c->stream));
  }
  const int limit = c->fixed_iters > 0 ? c->fixed_iters : c->U;
  const bool predicted = c->prev_iters > 0;
  int chunk = first_chunk(c, 0, limit);
  int enqueued = 0, misses = 0;
  for (;;) {
    if (chunk > 0) COFEM_TRY(run_cg_iterations(c, chunk));
    enqueued += chunk;
    int extra = 0;
    COFEM_TRY(poll_state(c, enqueued < limit, false, &extra));
    enqueued += extra;
    if (c->host_st->stop) break;
    if (enqueued > limit + 2) return fail(c, COFEM_ERR_DEVICE, "CG did not report completion after the iteration cap");
    chunk = next_chunk(c, predicted, ++misses, extra, enqueued, limit);
  }
  if (c->host_st->numeric_error)
    return fail(c, COFEM_ERR_NUMERIC, "non-finite value in a CG scalar at EM iteration " + std::to_string(t));
  const int iters = c->host_st->iter;
  // the solve's ratio against ||B||_F
  const double ratio = c->host_st->ratio * (warm ? c->tol / (tol_eff > 0.0 ? tol_eff : c->tol) : 1.0);
  if (warm) {
    double tol = c->tol;  // restore the solve's own tolerance for the next E-step's cold start
    COFEM_HIP(c, hipMemcpyAsync(&c->st->tol, &tol, sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  COFEM_HIP(c, dense_ir_accumulate(dd, c->Xt, c->X, c->xtm, c->xm, c->stream));
  if (c->true_resid) {
    COFEM_TRY(mark(c, COFEM_KT_CHECK, 0));
    COFEM_HIP(c, dense_pass1(dd, c->phiA, c->Xt, c->xtm, c->Wpart, c->wmpart, c->W, c->wm, c->cnt_split1, c->st, 1,
                             c->stream));
    COFEM_HIP(c, dense_pass2(dd, c->phiB, c->W, c->wm, c->Xt, c->xtm, c->R, c->rm, c->alpha, c->beta, c->Qpart,
                             c->qmpart, c->Qs, c->Qsm, c->parts_pass, c->cnts_pass, c->cnt_split2, c->st, 1,
                             c->stream));
    // ||B - A X||_F / ||B||_F: the true-residual sums use nB, which the warm
    // start moved to ||R0||_F; the ratio is rescaled below
    COFEM_HIP(c, dense_true_resid(dd, c->seed, t, c->K, c->b0, c->Qs, c->Qsm, c->parts_upd, c->cnts_upd, c->st,
                                  c->stream));
  }
  COFEM_TRY(mark(c, COFEM_KT_MSTEP, 0));
  COFEM_HIP(c, dense_mstep(dd, c->seed, t, c->K, c->Xt, c->xtm, c->alpha, c->alpha_max, c->mu, c->sdiag,
                           c->parts_upd, c->cnts_upd, c->st, c->stream));
  COFEM_TRY(mark(c, -1, 0));
  COFEM_TRY(iter_end(c));
  COFEM_TRY(read_state(c));
  COFEM_TRY(collect_times(c, iters));
  c->has_solution = true;
  c->prev_iters = iters;
  c->t_next = t + 1;
  if (out) {
    float ms = 0.0f;
    COFEM_TRY(iter_ms(c, &ms));
    const double nB0 = c->host_st->nB0, nB = c->host_st->nB;
    out->t = t;
    out->cg_iters = iters;
    out->converged = ratio < c->tol ? 1 : 0;
    out->n_clamped = c->host_st->n_clamped;
    out->rel_resid = ratio;
    out->ms = ms;
    out->rel_resid_true = c->true_resid ? c->host_st->true_ratio * (nB0 > 0.0 ? nB / nB0 : 1.0) : -1.0;
    out->ir_sweeps = 0;
    out->gamma_change = c->host_st->gamma_change;
  }
  return COFEM_OK;
}

// The plain EM iteration in three parts, so that a run of EM iterations can
// enqueue the start of the next one before it waits for the end of this one
// (the GPU then runs that start while the host reads this one's results):
// em_begin (iteration clock, the solve's start), em_solve (CG with its polls,
// the final checks, the M-step, an asynchronous copy of the state) and
// em_finish (waits for that copy; kernel times and statistics).
struct EmPending {
  int iters = 0;           // the solve's CG count
  size_t marks = 0;        // timing marks of this iteration (the first ones recorded)
  hipEvent_t e0 = nullptr; // the iteration's start event
  double t0_host = 0.0;
};

// `keep_marks`: timing marks of an earlier iteration are still to be read.
cofem_status em_begin(cofem_ctx* c, bool keep_marks) {
  const int t = c->t_next;
  COFEM_TRY(iter_start(c));
  c->cg_enq = 0;
  if (!keep_marks) c->kev_used = 0;
  COFEM_TRY(mark(c, COFEM_KT_INIT, 0));
  if (c->kind == COFEM_DENSE) {
    COFEM_TRY(dense_set_minv(c));
    COFEM_HIP(c, dense_init(c->dd, c->seed, t, c->K, c->b0, c->X, c->R, c->P, c->xm, c->rm, c->pm,
                            c->parts_init, c->cnts_init, c->st, c->stream, c->active_minv));
  }
  else if (conv_pcg(c)) {
    COFEM_TRY(conv_start_pcg(c, t));
  } else {
    COFEM_HIP(c, conv_init(c->cd, c->seed, t, c->b0, c->vX, c->vR, c->vP, c->xm, c->rm, c->pm, c->red_init,
                           c->st, c->stream));
  }
  return COFEM_OK;
}

cofem_status em_solve(cofem_ctx* c, EmPending* pd) {
  const int t = c->t_next;
  // launches per solve: conv needs one more than its updates (the first
  // operator pass)
  const int folded = folded_update(c) ? 1 : 0;
  const int limit = (c->fixed_iters > 0 ? c->fixed_iters : c->U) + folded;
  const bool predicted = c->prev_iters > 0;
  // where the previous count predicts the stop at the first poll, the launch
  // ahead of it is the true residual itself (persistent conv kernel): no idle
  // round trip between the solve and the residual
  const bool spec_resid = predicted && c->true_resid && c->kind == COFEM_CONV2D_CIRC && c->cd.ws_grid > 0;
  bool resid_done = false;
  int chunk = first_chunk(c, folded, limit);
  int enqueued = 0, misses = 0;
  for (;;) {
    if (chunk > 0) COFEM_TRY(run_cg_iterations(c, chunk));
    enqueued += chunk;
    int extra = 0;
    const bool spec = spec_resid && misses == 0;
    COFEM_TRY(poll_state(c, enqueued < limit, false, &extra, spec ? t : -1));
    enqueued += extra;
    if (c->host_st->stop) {
      resid_done = spec;
      break;
    }
    if (enqueued > limit + 2)
      return fail(c, COFEM_ERR_DEVICE, "CG did not report completion after the iteration cap");
    chunk = next_chunk(c, predicted, ++misses, extra, enqueued, limit);
  }
  if (c->host_st->numeric_error)
    return fail(c, COFEM_ERR_NUMERIC, "non-finite value in a CG scalar at EM iteration " + std::to_string(t));
  const int iters = c->host_st->iter;  // launches after the stop return at once
  if (c->true_resid && !resid_done) COFEM_TRY(true_residual(c, t));
  COFEM_TRY(mark(c, COFEM_KT_MSTEP, 0));
  if (c->kind == COFEM_DENSE)
    COFEM_HIP(c, dense_mstep(c->dd, c->seed, t, c->K, c->X, c->xm, c->alpha, c->alpha_max, c->mu,
                             c->sdiag, c->parts_upd, c->cnts_upd, c->st, c->stream));
  else {
    // the learned form's features see how far this M-step moves alpha: the
    // M-step keeps the old alpha in alpha_prev as it replaces it
    COFEM_HIP(c, conv_mstep(c->cd, c->seed, t, c->vX, c->xm, c->alpha, c->alpha_max, c->mu, c->sdiag,
                            c->red_upd, c->st, c->stream, c->alpha_prev));
  }
  c->alpha_uniform = false;
  COFEM_TRY(mark(c, -1, 0));
  COFEM_TRY(iter_end(c));
  CgScalars* end = c->host_end ? c->host_end : c->host_st;
  COFEM_HIP(c, hipMemcpyAsync(end, c->st, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
  if (c->ev_end) COFEM_HIP(c, hipEventRecord(c->ev_end, c->stream));
  pd->iters = iters;
  pd->marks = c->kev_used;
  pd->e0 = c->ev0;
  pd->t0_host = c->t0_host;
  c->has_solution = true;
  c->prev_iters = iters;
  c->t_next = t + 1;
  return COFEM_OK;
}

cofem_status em_finish(cofem_ctx* c, const EmPending& pd, int t, cofem_iter_stats* out) {
  if (c->ev_end)
    COFEM_HIP(c, hipEventSynchronize(c->ev_end));
  else
    COFEM_HIP(c, hipStreamSynchronize(c->stream));
  const CgScalars* end = c->host_end ? c->host_end : c->host_st;
  // (a conv solve of n updates has n + 1 working launches)
  COFEM_TRY(collect_times(c, pd.iters + (folded_update(c) ? 1 : 0), pd.marks));
  if (out) {
    float ms = 0.0f;
    if (pd.e0 && c->ev1)
      COFEM_HIP(c, hipEventElapsedTime(&ms, pd.e0, c->ev1));
    else
      ms = (float)(host_ms() - pd.t0_host);
    out->t = t;
    out->cg_iters = end->iter;
    out->converged = end->ratio < c->tol ? 1 : 0;
    out->n_clamped = end->n_clamped;
    out->rel_resid = end->ratio;
    out->ms = ms;
    out->rel_resid_true = c->true_resid ? end->true_ratio : -1.0;
    out->ir_sweeps = 0;
    out->gamma_change = end->gamma_change;
    if (c->per_col) out->converged = end->all_done;
  }
  return COFEM_OK;
}

// Whether an EM iteration takes the plain path (em_begin / em_solve / em_finish).
bool plain_em(const cofem_ctx* c) {
  return !c->batch && c->precision != COFEM_PREC_BF16_IR &&
         !(c->kind == COFEM_DENSE && (c->flags & COFEM_FLAG_WARM_PREV));
}

cofem_status em_iteration(cofem_ctx* c, cofem_iter_stats* out) {
  if (c->batch) return em_iteration_batch(c, out);
  if (c->precision == COFEM_PREC_BF16_IR) return em_iteration_ir(c, out);
  if (c->kind == COFEM_DENSE && (c->flags & COFEM_FLAG_WARM_PREV)) return em_iteration_dense_warm(c, out);
  const int t = c->t_next;
  EmPending pd;
  COFEM_TRY(em_begin(c, false));
  COFEM_TRY(em_solve(c, &pd));
  return em_finish(c, pd, t, out);
}

// n EM iterations of the plain path, each one's start enqueued before the
// previous one's end is read.  The device work and its order are those of n
// calls of em_iteration; only the host waits move.
cofem_status em_iterations_pipelined(cofem_ctx* c, int n, cofem_iter_stats* stats) {
  if (n <= 0) return COFEM_OK;
  if (c->t_next >= (1 << 16)) return fail(c, COFEM_ERR_INVALID_ARG, "EM iteration index beyond 65535");
  COFEM_TRY(em_begin(c, false));
  for (int i = 0; i < n; ++i) {
    const int t = c->t_next;
    EmPending pd;
    COFEM_TRY(em_solve(c, &pd));
    cofem_status next = COFEM_OK;
    if (i + 1 < n) {
      if (c->t_next >= (1 << 16)) {
        next = fail(c, COFEM_ERR_INVALID_ARG, "EM iteration index beyond 65535");
      } else {
        // the next iteration's clock starts on the spare event: pd.e0 still
        // holds this one's start
        std::swap(c->ev0, c->ev0_alt);
        next = em_begin(c, true);
      }
    }
    COFEM_TRY(em_finish(c, pd, t, stats ? &stats[i] : nullptr));
    if (next != COFEM_OK) return next;
  }
  return COFEM_OK;
}

// The problem description and the solver controls of a context (no device
// state yet).
void setup_ctx(cofem_ctx* c, const cofem_problem* problems, const cofem_params* params, void* hip_stream) {
  const cofem_problem& p = problems[0];
  c->kind = p.kind;
  c->NT = p.n_tasks > 1 ? p.n_tasks : 1;  // validated: several tasks only for the DCT dictionary
  c->N = p.N;
  c->D = p.D;
  c->K = params->K;
  c->beta = params->beta;
  c->tol = params->cg_tol;
  c->U = params->cg_max_iter;
  c->seed = params->seed;
  c->alpha_max = params->alpha_max > 0.0 ? params->alpha_max : 1e10;
  c->poll = params->poll_interval > 0 ? params->poll_interval : 8;
  c->precision = params->precision;
  c->per_col = params->stop_rule == COFEM_STOP_PER_COLUMN;
  c->true_resid = (params->flags & COFEM_FLAG_TRUE_RESIDUAL) != 0;
  c->flags = params->flags;
  c->tol_in = params->ir_inner_tol > 0.0 ? params->ir_inner_tol : 0.1;
  c->max_sweeps = params->ir_max_sweeps > 0 ? params->ir_max_sweeps : 20;
  c->stream = static_cast<hipStream_t>(hip_stream);
}

cofem_ctx* new_ctx(const cofem_problem* problems, const cofem_params* params, void* hip_stream) {
  cofem_ctx* c = new (std::nothrow) cofem_ctx();
  if (c) setup_ctx(c, problems, params, hip_stream);
  return c;
}

// Allocates (or, when sizing, counts) the device state of every problem and
// sets it up.
cofem_status init_state(cofem_ctx* c, const cofem_problem* problems, int32_t n_problems, const cofem_params* params) {
  const cofem_problem& p = problems[0];
  const bool batched = n_problems > 1 || p.phi_dtype == COFEM_BF16 || (params->flags & COFEM_FLAG_BATCHED);
  COFEM_TRY(alloc(c, &c->st, (size_t)n_problems));
  return batched                      ? init_batch(c, problems, n_problems)
         : (p.kind == COFEM_DENSE)    ? init_dense(c, p)
         : (p.kind == COFEM_DCT_MASK) ? init_dct(c, p)
                                      : init_conv(c, p);
}

// Device memory of the allocation-free entry point (cofem_em_step_static): a
// file-scope array in the library's code object, kStaticScratchBytes on every
// GPU the library runs on, held until the process ends.  Host code must not
// pass `scratch` itself to a kernel or copy (on the host that name is only a
// stand-in); its device address comes from hipGetSymbolAddress, once per
// device with that device current, and is kept in g_scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

cofem_status static_scratch(int device, char** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(nullptr, COFEM_ERR_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, COFEM_ERR_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return COFEM_OK;
}

}  // namespace

extern "C" {

cofem_status cofem_workspace_size(const cofem_problem* problems, int32_t n_problems, const cofem_params* params,
                                  size_t* bytes) {
  if (!bytes) return fail(nullptr, COFEM_ERR_INVALID_ARG, "bytes is null");
  std::string why;
  cofem_status v = validate(problems, n_problems, params, &why);
  if (v != COFEM_OK) return fail(nullptr, v, why);
  cofem_ctx* c = new_ctx(problems, params, nullptr);
  if (!c) return fail(nullptr, COFEM_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->sizing = true;
  const cofem_status s = init_state(c, problems, n_problems, params);
  const size_t need = c->ws_used;
  if (s != COFEM_OK) g_err = c->err;
  delete c->batch;
  delete c;  // nothing was allocated or launched
  if (s != COFEM_OK) return s;
  *bytes = need;
  return COFEM_OK;
}

cofem_status cofem_init(const cofem_problem* problems, int32_t n_problems, const cofem_params* params,
                        void* hip_stream, void* workspace, size_t workspace_bytes, cofem_ctx** out) {
  if (!out) return fail(nullptr, COFEM_ERR_INVALID_ARG, "out is null");
  if (workspace && reinterpret_cast<uintptr_t>(workspace) % kWsAlign != 0)
    return fail(nullptr, COFEM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (!workspace && workspace_bytes != 0)
    return fail(nullptr, COFEM_ERR_INVALID_ARG, "workspace_bytes without a workspace");
  std::string why;
  cofem_status v = validate(problems, n_problems, params, &why);
  if (v != COFEM_OK) return fail(nullptr, v, why);
  cofem_ctx* c = new_ctx(problems, params, hip_stream);
  if (!c) return fail(nullptr, COFEM_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->ws = static_cast<char*>(workspace);
  c->ws_size = workspace ? workspace_bytes : 0;
  cofem_status s = COFEM_OK;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_state, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_end, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&c->ev0_alt);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->host_st), 2 * sizeof(CgScalars));
  if (e == hipSuccess) c->host_end = c->host_st + 1;
  if (e != hipSuccess) {
    s = fail(c, COFEM_ERR_DEVICE, std::string("HIP set-up: ") + hipGetErrorString(e));
  }
  if (s == COFEM_OK) s = init_state(c, problems, n_problems, params);
  if (s == COFEM_OK) s = push_controls(c);
  if (s == COFEM_OK) {
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = fail(c, COFEM_ERR_DEVICE, std::string("init: ") + hipGetErrorString(e));
  }
  if (s != COFEM_OK) {
    g_err = c->err;
    destroy_ctx(c);
    return s;
  }
  *out = c;
  return COFEM_OK;
}

cofem_status cofem_em_step_static(const cofem_problem* problem, const cofem_params* params, const float* alpha_in,
                                  int32_t t, float* mu, float* s, float* alpha_out, cofem_iter_stats* stats,
                                  void* hip_stream) {
  std::string why;
  cofem_status v = validate(problem, 1, params, &why);
  if (v != COFEM_OK) return fail(nullptr, v, why);
  if (problem->phi_dtype != COFEM_F32 || (params->flags & (COFEM_FLAG_BATCHED | COFEM_FLAG_EAGER)))
    return fail(nullptr, COFEM_ERR_UNSUPPORTED, "the allocation-free step takes one float32 problem (no batched form)");
  if (params->precision == COFEM_PREC_BF16_IR)
    return fail(nullptr, COFEM_ERR_UNSUPPORTED, "the allocation-free step runs COFEM_PREC_FP32 or COFEM_PREC_FP64");
  if (params->flags & COFEM_FLAG_WARM_PREV)
    return fail(nullptr, COFEM_ERR_UNSUPPORTED, "a single stateless step has no previous E-step to start from");
  if (params->flags & COFEM_FLAG_SPECTRAL_START)
    return fail(nullptr, COFEM_ERR_UNSUPPORTED, "the allocation-free step takes any alpha: no spectral start");
  if (!alpha_in) return fail(nullptr, COFEM_ERR_INVALID_ARG, "alpha_in is null");
  if (t < 0 || t >= (1 << 16)) return fail(nullptr, COFEM_ERR_INVALID_ARG, "t must be in [0, 65535]");
  // the layout this problem needs, counted without touching the device
  size_t need = 0;
  {
    cofem_ctx sz;
    setup_ctx(&sz, problem, params, hip_stream);
    sz.sizing = true;
    const cofem_status st = init_state(&sz, problem, 1, params);
    delete sz.batch;
    sz.batch = nullptr;
    if (st != COFEM_OK) return fail(nullptr, st, sz.err);
    need = sz.ws_used;
  }
  if (need > kStaticScratchBytes)
    return fail(nullptr, COFEM_ERR_INVALID_ARG,
                "the problem needs " + std::to_string(need) + " bytes of device memory; the static scratch holds " +
                    std::to_string(kStaticScratchBytes));
  cofem_ctx c;
  setup_ctx(&c, problem, params, hip_stream);
  CgScalars host_state;  // pageable: the state reads are synchronous copies
  c.host_st = &host_state;
  COFEM_HIP(&c, hipGetDevice(&c.device));
  COFEM_TRY(static_scratch(c.device, &c.ws));
  c.ws_size = kStaticScratchBytes;
  cofem_status st = init_state(&c, problem, 1, params);
  if (st == COFEM_OK) st = push_controls(&c);
  if (st == COFEM_OK) st = cofem_set_alpha(&c, 0, alpha_in);
  if (st == COFEM_OK) {
    c.t_next = t;
    cofem_iter_stats local;
    st = em_iteration(&c, stats ? stats : &local);
  }
  if (st == COFEM_OK) st = cofem_posterior(&c, 0, mu, s, alpha_out);
  if (st == COFEM_OK) {
    const hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) st = fail(&c, COFEM_ERR_DEVICE, std::string("static step: ") + hipGetErrorString(e));
  }
  if (st != COFEM_OK) g_err = c.err;
  return st;
}

cofem_status cofem_em_step(cofem_ctx* ctx, int32_t n_iters, cofem_iter_stats* stats) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (n_iters < 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "n_iters < 0");
  if (plain_em(ctx) && ctx->ev_end && ctx->ev0_alt && ctx->host_end) {
    const cofem_status s = em_iterations_pipelined(ctx, n_iters, stats);
    // a failed E-step may leave non-finite iterates: no later solve starts there
    if (s != COFEM_OK) forget_solution(ctx);
    return s;
  }
  for (int i = 0; i < n_iters; ++i) {
    if (ctx->t_next >= (1 << 16)) return fail(ctx, COFEM_ERR_INVALID_ARG, "EM iteration index beyond 65535");
    const int np = ctx->batch ? ctx->batch->n : 1;
    const cofem_status s = em_iteration(ctx, stats ? &stats[(size_t)i * np] : nullptr);
    if (s != COFEM_OK) {
      // a failed E-step may leave non-finite iterates: no later solve starts there
      forget_solution(ctx);
      return s;
    }
  }
  return COFEM_OK;
}

cofem_status cofem_em_run(cofem_ctx* ctx, int32_t max_iters, double em_tol, cofem_iter_stats* stats,
                          int32_t* n_done) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (max_iters < 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "max_iters < 0");
  if (!(em_tol == em_tol)) return fail(ctx, COFEM_ERR_INVALID_ARG, "em_tol is NaN");
  const int np = ctx->batch ? ctx->batch->n : 1;
  std::vector<cofem_iter_stats> one((size_t)np);
  int done = 0;
  for (int i = 0; i < max_iters; ++i) {
    if (ctx->t_next >= (1 << 16)) return fail(ctx, COFEM_ERR_INVALID_ARG, "EM iteration index beyond 65535");
    cofem_iter_stats* out = stats ? &stats[(size_t)i * np] : one.data();
    const cofem_status s = em_iteration(ctx, out);
    if (s != COFEM_OK) {
      forget_solution(ctx);
      return s;
    }
    ++done;
    bool small = em_tol > 0.0;
    for (int j = 0; j < np && small; ++j) small = out[j].gamma_change < em_tol;
    if (small) break;
  }
  if (n_done) *n_done = done;
  return COFEM_OK;
}

cofem_status cofem_posterior(cofem_ctx* ctx, int32_t problem, float* mu, float* s, float* alpha) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  const int np = ctx->batch ? ctx->batch->n : 1;
  if (problem < 0 || problem >= np) return fail(ctx, COFEM_ERR_INVALID_ARG, "problem index out of range");
  const float *pmu = ctx->mu, *ps = ctx->sdiag, *pa = ctx->alpha;
  int64_t D = ctx->D;
  if (ctx->batch) {
    const BatchProblem& p = ctx->batch->probs[problem];
    pmu = p.mu;
    ps = p.sdiag;
    pa = p.alpha;
    D = p.D;
  }
  if (ctx->kind == COFEM_DCT_MASK) {
    // state order -> natural coefficient order
    if (mu) COFEM_HIP(ctx, perm_out_f32(ctx->cd, pmu, mu, ctx->stream));
    if (s) COFEM_HIP(ctx, perm_out_f32(ctx->cd, ps, s, ctx->stream));
    if (alpha) COFEM_HIP(ctx, perm_out_f32(ctx->cd, pa, alpha, ctx->stream));
    return COFEM_OK;
  }
  const size_t bytes = sizeof(float) * (size_t)D;
  if (mu) COFEM_HIP(ctx, hipMemcpyAsync(mu, pmu, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (s) COFEM_HIP(ctx, hipMemcpyAsync(s, ps, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (alpha) COFEM_HIP(ctx, hipMemcpyAsync(alpha, pa, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  return COFEM_OK;
}

cofem_status cofem_set_alpha(cofem_ctx* ctx, int32_t problem, const float* alpha) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  const int np = ctx->batch ? ctx->batch->n : 1;
  if (problem < 0 || problem >= np) return fail(ctx, COFEM_ERR_INVALID_ARG, "problem index out of range");
  if (!alpha) return fail(ctx, COFEM_ERR_INVALID_ARG, "alpha is null");
  float* dst = ctx->batch ? ctx->batch->probs[problem].alpha : ctx->alpha;
  const int64_t D = ctx->batch ? ctx->batch->probs[problem].D : ctx->D;
  ctx->alpha_uniform = false;  // not inspected: the spectral start waits for cofem_restart
  if (ctx->kind == COFEM_DCT_MASK)
    COFEM_HIP(ctx, perm_in_f32(ctx->cd, alpha, dst, ctx->stream));
  else
    COFEM_HIP(ctx, hipMemcpyAsync(dst, alpha, sizeof(float) * (size_t)D, hipMemcpyDeviceToDevice, ctx->stream));
  return COFEM_OK;
}

cofem_status cofem_get_means(cofem_ctx* ctx, int32_t problem, double* mu) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (!mu) return fail(ctx, COFEM_ERR_INVALID_ARG, "mu is null");
  if (ctx->batch || ctx->NT == 1) {
    // one task: the mean column of the solution
    return cofem_get_solution(ctx, problem, nullptr, mu);
  }
  if (problem != 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "problem index out of range");
  // task t's column sits at t * ldD (ldD = D for the DCT dictionary, Dp for a dense one)
  const int64_t ld = ctx->kind == COFEM_DENSE ? ctx->dd.Dp : ctx->cd.ldD;
  for (int t = 0; t < ctx->NT; ++t) {
    const double* src = ctx->xm + (size_t)t * ld;
    double* dst = mu + (size_t)t * ctx->D;
    if (ctx->kind == COFEM_DCT_MASK)
      COFEM_HIP(ctx, perm_out_f64(ctx->cd, src, dst, ctx->stream));
    else
      COFEM_HIP(ctx, hipMemcpyAsync(dst, src, sizeof(double) * (size_t)ctx->D, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return COFEM_OK;
}

cofem_status cofem_set_iteration(cofem_ctx* ctx, int32_t t) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (t < 0 || t >= (1 << 16)) return fail(ctx, COFEM_ERR_INVALID_ARG, "t must be in [0, 65535]");
  ctx->t_next = t;
  // the last solve no longer precedes the next E-step: start it cold
  forget_solution(ctx);
  return COFEM_OK;
}

cofem_status cofem_restart(cofem_ctx* ctx) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  forget_solution(ctx);
  ctx->t_next = 1;
  ctx->prev_iters = ctx->fixed_iters;
  if (BatchHost* b = ctx->batch) {
    for (const BatchProblem& p : b->probs) {
      COFEM_HIP(ctx, fill_f32(p.alpha, 1.0f, p.Dp, ctx->stream));
      COFEM_HIP(ctx, fill_f32(p.mu, 0.0f, p.Dp, ctx->stream));
      COFEM_HIP(ctx, fill_f32(p.sdiag, 0.0f, p.Dp, ctx->stream));
    }
    return COFEM_OK;
  }
  const int64_t n = ctx->kind == COFEM_DENSE ? ctx->dd.Dp : ctx->cd.ldD;
  COFEM_HIP(ctx, fill_f32(ctx->alpha, 1.0f, n, ctx->stream));
  ctx->alpha_uniform = true;
  ctx->alpha_a0 = 1.0;
  if (ctx->alpha_prev) COFEM_HIP(ctx, fill_f32(ctx->alpha_prev, 1.0f, n, ctx->stream));
  COFEM_HIP(ctx, fill_f32(ctx->mu, 0.0f, n, ctx->stream));
  COFEM_HIP(ctx, fill_f32(ctx->sdiag, 0.0f, n, ctx->stream));
  return COFEM_OK;
}

cofem_status cofem_set_fixed_cg_iters(cofem_ctx* ctx, int32_t n) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (ctx->precision == COFEM_PREC_BF16_IR)
    return fail(ctx, COFEM_ERR_UNSUPPORTED, "fixed CG counts are not available under COFEM_PREC_BF16_IR");
  if (n < 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "n must be >= 0");
  ctx->fixed_iters = n;
  ctx->prev_iters = n;
  return push_controls(ctx);
}

cofem_status cofem_get_solution(cofem_ctx* ctx, int32_t problem, float* probes, double* mean) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (ctx->batch) {
    if (problem < 0 || problem >= ctx->batch->n) return fail(ctx, COFEM_ERR_INVALID_ARG, "problem index out of range");
    const BatchProblem& p = ctx->batch->probs[problem];
    if (probes) COFEM_HIP(ctx, dense_to_colmajor(ctx->batch->dims[problem], ctx->K, p.X, probes, ctx->stream));
    if (mean)
      COFEM_HIP(ctx, hipMemcpyAsync(mean, p.xm, sizeof(double) * (size_t)p.D, hipMemcpyDeviceToDevice, ctx->stream));
    return COFEM_OK;
  }
  if (problem != 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "problem index out of range");
  // dense forms that accumulate the solution (refinement, warm start) keep it in Xt
  const bool ir = ctx->kind == COFEM_DENSE && ctx->Xt != nullptr;
  if (probes) {
    if (ctx->kind == COFEM_DENSE) {
      COFEM_HIP(ctx, dense_to_colmajor(ctx->dd, ctx->K, ir ? ctx->Xt : ctx->X, probes, ctx->stream));
    } else {
      COFEM_HIP(ctx, conv_probes_out(ctx->cd, ctx->vX, probes, ctx->stream));
    }
  }
  if (mean && ctx->kind == COFEM_DCT_MASK)
    COFEM_HIP(ctx, perm_out_f64(ctx->cd, ctx->xm, mean, ctx->stream));
  else if (mean)
    COFEM_HIP(ctx, hipMemcpyAsync(mean, ir ? ctx->xtm : ctx->xm, sizeof(double) * (size_t)ctx->D,
                                  hipMemcpyDeviceToDevice, ctx->stream));
  return COFEM_OK;
}

static cofem_status apply_A_impl(cofem_ctx* ctx, int32_t problem, const float* v_probes, const double* v_mean,
                                 float* q_probes, double* q_mean, bool lowp) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (problem != 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "problem index out of range");
  if (!v_probes || !v_mean || !q_probes || !q_mean) return fail(ctx, COFEM_ERR_INVALID_ARG, "null vector");
  if (ctx->batch) return fail(ctx, COFEM_ERR_UNSUPPORTED, "operator application is not built for the batched form");
  if (lowp && ctx->precision != COFEM_PREC_BF16_IR)
    return fail(ctx, COFEM_ERR_UNSUPPORTED, "the low-precision operator exists only under COFEM_PREC_BF16_IR");
  const size_t Dm = sizeof(double) * (size_t)ctx->D;
  if (ctx->kind == COFEM_DENSE) {
    const DenseDims& dd = ctx->dd;
    COFEM_HIP(ctx, dense_from_colmajor(dd, ctx->K, v_probes, ctx->Vs, ctx->stream));
    COFEM_HIP(ctx, hipMemsetAsync(ctx->Vsm, 0, sizeof(double) * dd.Dp, ctx->stream));
    COFEM_HIP(ctx, hipMemcpyAsync(ctx->Vsm, v_mean, Dm, hipMemcpyDeviceToDevice, ctx->stream));
    if (lowp) {
      COFEM_HIP(ctx, dense16_pass1(dd, ctx->phiA16, ctx->Vs, ctx->Vsm, ctx->Wpart, ctx->wmpart, ctx->W, ctx->wm,
                                   ctx->cnt_split1, ctx->st, 1, ctx->stream));
      COFEM_HIP(ctx, dense16_pass2(dd, ctx->phiB16, ctx->W, ctx->wm, ctx->Vs, ctx->Vsm, ctx->Vs, ctx->Vsm,
                                   ctx->alpha, ctx->beta, ctx->Qpart, ctx->qmpart, ctx->Qs, ctx->Qsm,
                                   ctx->parts_pass, ctx->cnts_pass, ctx->cnt_split2, ctx->st, 1, ctx->stream));
    } else {
      COFEM_HIP(ctx, dense_pass1(dd, ctx->phiA, ctx->Vs, ctx->Vsm, ctx->Wpart, ctx->wmpart, ctx->W, ctx->wm,
                                 ctx->cnt_split1, ctx->st, 1, ctx->stream));
      COFEM_HIP(ctx, dense_pass2(dd, ctx->phiB, ctx->W, ctx->wm, ctx->Vs, ctx->Vsm, ctx->Vs, ctx->Vsm,
                                 ctx->alpha, ctx->beta, ctx->Qpart, ctx->qmpart, ctx->Qs, ctx->Qsm,
                                 ctx->parts_pass, ctx->cnts_pass, ctx->cnt_split2, ctx->st, 1, ctx->stream));
    }
    COFEM_HIP(ctx, dense_to_colmajor(dd, ctx->K, ctx->Qs, q_probes, ctx->stream));
  } else if (ctx->kind == COFEM_DCT_MASK) {
    const ConvDims& cd = ctx->cd;
    COFEM_HIP(ctx, conv_probes_in(cd, v_probes, ctx->vVs, ctx->stream));
    COFEM_HIP(ctx, perm_in_f64(cd, v_mean, ctx->Vsm, ctx->stream));
    COFEM_HIP(ctx, dct_rows_in(ctx->xd, ctx->xb, nullptr, nullptr, ctx->vVs, nullptr, nullptr, nullptr, ctx->Vsm,
                               nullptr, nullptr, ctx->st, 0, 1, ctx->stream));
    COFEM_HIP(ctx, dct_mid(ctx->xd, ctx->xb, ctx->st, 1, ctx->stream));
    COFEM_HIP(ctx, dct_rows_out(ctx->xd, ctx->xb, ctx->vVs, nullptr, ctx->vQs, ctx->Vsm, nullptr, ctx->Qsm,
                                ctx->alpha, nullptr, ctx->red_pass, ctx->st, 0, 1, ctx->stream));
    COFEM_HIP(ctx, conv_probes_out(cd, ctx->vQs, q_probes, ctx->stream));
    COFEM_HIP(ctx, perm_out_f64(cd, ctx->Qsm, q_mean, ctx->stream));
    COFEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return COFEM_OK;
  } else {
    const ConvDims& cd = ctx->cd;
    COFEM_HIP(ctx, conv_probes_in(cd, v_probes, ctx->vVs, ctx->stream));
    COFEM_HIP(ctx, hipMemcpyAsync(ctx->Vsm, v_mean, Dm, hipMemcpyDeviceToDevice, ctx->stream));
    COFEM_HIP(ctx, conv_pass(cd, ctx->taps, ctx->vVs, ctx->Vsm, ctx->vVs, ctx->Vsm, ctx->alpha, ctx->beta,
                             ctx->vQs, ctx->Qsm, ctx->red_pass, ctx->st, 1, ctx->stream));
    COFEM_HIP(ctx, conv_probes_out(cd, ctx->vQs, q_probes, ctx->stream));
  }
  COFEM_HIP(ctx, hipMemcpyAsync(q_mean, ctx->Qsm, Dm, hipMemcpyDeviceToDevice, ctx->stream));
  COFEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return COFEM_OK;
}

cofem_status cofem_apply_A(cofem_ctx* ctx, int32_t problem, const float* v_probes, const double* v_mean,
                           float* q_probes, double* q_mean) {
  return apply_A_impl(ctx, problem, v_probes, v_mean, q_probes, q_mean, false);
}

cofem_status cofem_apply_A_lowp(cofem_ctx* ctx, int32_t problem, const float* v_probes, const double* v_mean,
                                float* q_probes, double* q_mean) {
  return apply_A_impl(ctx, problem, v_probes, v_mean, q_probes, q_mean, true);
}

cofem_status cofem_get_ir_sweeps(cofem_ctx* ctx, int32_t* counts, int32_t capacity, int32_t* n) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (!n || capacity < 0 || (capacity > 0 && !counts)) return fail(ctx, COFEM_ERR_INVALID_ARG, "bad output");
  if (ctx->precision != COFEM_PREC_BF16_IR)
    return fail(ctx, COFEM_ERR_UNSUPPORTED, "refinement sweeps exist only under COFEM_PREC_BF16_IR");
  const int32_t m = (int32_t)ctx->sweeps.size();
  for (int32_t i = 0; i < m && i < capacity; ++i) counts[i] = ctx->sweeps[i];
  *n = m;
  return COFEM_OK;
}

cofem_status cofem_probe_signs(uint64_t seed, int32_t t, int32_t K, int64_t D, float* out, void* hip_stream) {
  if (!out) return fail(nullptr, COFEM_ERR_INVALID_ARG, "out is null");
  if (t < 0 || t >= (1 << 16) || K < 0 || K > (1 << 16) || D < 0 || D >= ((int64_t)1 << 38))
    return fail(nullptr, COFEM_ERR_INVALID_ARG, "probe index out of range");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = probe_signs_colmajor(seed, t, K, D, out, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(nullptr, COFEM_ERR_DEVICE, std::string("probe kernel: ") + hipGetErrorString(e));
  return COFEM_OK;
}

cofem_status cofem_time_operator(cofem_ctx* ctx, int32_t reps, float* ms_out) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (reps < 1 || !ms_out) return fail(ctx, COFEM_ERR_INVALID_ARG, "reps < 1 or ms_out null");
  if (BatchHost* b = ctx->batch) {
    // grouped passes over every problem, apply only, back to back
    float ms[2] = {0.f, 0.f};
    for (int k = 0; k < 2; ++k) {
      auto launch = [&]() {
        return k == 0 ? batch_pass1(b->d_items1, b->n1, b->d_probs, 1, ctx->stream)
                      : batch_pass2(b->d_items2, b->n2, b->d_probs, ctx->beta, 1, ctx->stream);
      };
      COFEM_HIP(ctx, launch());
      COFEM_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
      for (int r = 0; r < reps; ++r) COFEM_HIP(ctx, launch());
      COFEM_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
      COFEM_HIP(ctx, hipEventSynchronize(ctx->ev1));
      COFEM_HIP(ctx, hipEventElapsedTime(&ms[k], ctx->ev0, ctx->ev1));
    }
    ms_out[0] = ms[0] / (float)reps;
    ms_out[1] = ms[1] / (float)reps;
    ms_out[2] = 0.f;
    return COFEM_OK;
  }
  // Each pass is launched `reps` times back to back between one pair of
  // events, as the CG loop issues them, so the average is the kernel's
  // duration plus the dispatch gap, not the latency of an isolated launch.
  auto timed = [&](auto launch, float* out) -> cofem_status {
    COFEM_HIP(ctx, launch());  // warm
    COFEM_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    for (int r = 0; r < reps; ++r) COFEM_HIP(ctx, launch());
    COFEM_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    COFEM_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    COFEM_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    *out = ms / (float)reps;
    return COFEM_OK;
  };
  ms_out[0] = ms_out[1] = ms_out[2] = 0.f;
  cofem_status rc;
  if (ctx->kind == COFEM_DENSE) {
    rc = timed([&] { return dense_pass1(ctx->dd, ctx->phiA, ctx->P, ctx->pm, ctx->Wpart, ctx->wmpart, ctx->W,
                                        ctx->wm, ctx->cnt_split1, ctx->st, 1, ctx->stream); },
               &ms_out[0]);
    if (rc != COFEM_OK) return rc;
    rc = timed([&] { return dense_pass2(ctx->dd, ctx->phiB, ctx->W, ctx->wm, ctx->P, ctx->pm, ctx->R, ctx->rm,
                                        ctx->alpha, ctx->beta, ctx->Qpart, ctx->qmpart, ctx->Qs, ctx->Qsm,
                                        ctx->parts_pass, ctx->cnts_pass, ctx->cnt_split2, ctx->st, 1,
                                        ctx->stream); },
               &ms_out[1]);
  } else if (ctx->kind == COFEM_DCT_MASK) {
    const DctDims& xd = ctx->xd;
    const DctBuffers& xb = ctx->xb;
    rc = timed([&] { return dct_rows_in(xd, xb, nullptr, nullptr, ctx->vP, nullptr, nullptr, nullptr, ctx->pm,
                                        nullptr, nullptr, ctx->st, 0, 1, ctx->stream); },
               &ms_out[0]);
    if (rc != COFEM_OK) return rc;
    rc = timed([&] { return dct_mid(xd, xb, ctx->st, 1, ctx->stream); }, &ms_out[1]);
    if (rc != COFEM_OK) return rc;
    rc = timed([&] { return dct_rows_out(xd, xb, ctx->vP, nullptr, ctx->vQs, ctx->pm, nullptr, ctx->Qsm,
                                         ctx->alpha, nullptr, ctx->red_pass, ctx->st, 0, 1, ctx->stream); },
               &ms_out[2]);
  } else {
    rc = timed([&] { return conv_pass(ctx->cd, ctx->taps, ctx->vP, ctx->pm, ctx->vR, ctx->rm, ctx->alpha,
                                      ctx->beta, ctx->vQs, ctx->Qsm, ctx->red_pass, ctx->st, 1, ctx->stream); },
               &ms_out[0]);
  }
  return rc;
}

cofem_status cofem_set_kernel_timing(cofem_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (enable < 0) return fail(ctx, COFEM_ERR_INVALID_ARG, "kernel timing period must be >= 0");
  ctx->ktime = enable != 0;
  ctx->kt_every = enable > 0 ? enable : 1;
  ctx->kt_seq = 0;
  ctx->kev_used = 0;
  for (int i = 0; i < COFEM_KT_SLOTS; ++i) {
    ctx->kt_ms[i] = 0.0;
    ctx->kt_n[i] = 0;
  }
  return COFEM_OK;
}

cofem_status cofem_get_kernel_timing(cofem_ctx* ctx, double* ms_total, int64_t* launches) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (!ms_total || !launches) return fail(ctx, COFEM_ERR_INVALID_ARG, "null output array");
  for (int i = 0; i < COFEM_KT_SLOTS; ++i) {
    ms_total[i] = ctx->kt_ms[i];
    launches[i] = ctx->kt_n[i];
  }
  return COFEM_OK;
}

const char* cofem_kernel_name(const cofem_ctx* ctx, int32_t slot) {
  if (!ctx || (slot != COFEM_KT_PASS1 && slot != COFEM_KT_PASS2)) return nullptr;
  const bool p1 = slot == COFEM_KT_PASS1;
  if (ctx->kind == COFEM_DENSE) {
    if (ctx->precision == COFEM_PREC_BF16_IR) return p1 ? "k_dense16_pass1" : "k_dense16_pass2";
    return p1 ? "k_dense_pass1" : "k_dense_pass2";
  }
  if (ctx->kind == COFEM_DCT_MASK) return p1 ? "k_dct_rows_in" : "k_dct_mid";
  if (ctx->cd.ws_grid > 0) return "k_conv_ws";
  return p1 ? "k_conv_fused" : "k_conv_pass";
}

cofem_status cofem_batch_plan(cofem_ctx* ctx, int32_t* target_wgs, float* candidate_ms, int32_t* splits1,
                              int32_t* splits2) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (!ctx->batch) return fail(ctx, COFEM_ERR_UNSUPPORTED, "not a batched context");
  const BatchHost* b = ctx->batch;
  if (target_wgs) *target_wgs = b->target;
  if (candidate_ms)
    for (int k = 0; k < 4; ++k) candidate_ms[k] = b->cand_ms[k];
  for (int i = 0; i < b->n; ++i) {
    if (splits1) splits1[i] = b->probs[i].S1;
    if (splits2) splits2[i] = b->probs[i].S2;
  }
  return COFEM_OK;
}

cofem_status cofem_features(cofem_ctx* ctx, cofem_net* net, float* feats, float* aux) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (!net || !feats || !aux) return fail(ctx, COFEM_ERR_INVALID_ARG, "null net or output");
  if (ctx->kind != COFEM_CONV2D_CIRC || ctx->batch)
    return fail(ctx, COFEM_ERR_UNSUPPORTED, "features exist for convolution dictionaries only");
  if (net_height(net) != ctx->cd.H || net_width(net) != ctx->cd.W)
    return fail(ctx, COFEM_ERR_INVALID_ARG, "the net's image size differs from the problem's");
  COFEM_TRY(net_features(net, ctx->alpha, ctx->alpha_prev, ctx->xm, ctx->sdiag, ctx->taps, ctx->cd.ks * ctx->cd.ks,
                         ctx->beta, feats, aux, ctx->stream));
  COFEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return COFEM_OK;
}

cofem_status cofem_set_predictor(cofem_ctx* ctx, cofem_net* net) {
  if (!ctx) return fail(nullptr, COFEM_ERR_INVALID_ARG, "ctx is null");
  if (ctx->kind != COFEM_CONV2D_CIRC || ctx->batch)
    return fail(ctx, COFEM_ERR_UNSUPPORTED, "the learned form is built for convolution dictionaries");
  if (net && ctx->NT > 1)
    return fail(ctx, COFEM_ERR_UNSUPPORTED, "the learned form predicts one mean: single-task contexts only");
  if (net && (net_height(net) != ctx->cd.H || net_width(net) != ctx->cd.W))
    return fail(ctx, COFEM_ERR_INVALID_ARG, "the net's image size differs from the problem's");
  ctx->predictor = net ? predictor_hook : nullptr;
  ctx->predictor_user = net;
  return COFEM_OK;
}

void cofem_destroy(cofem_ctx* ctx) { destroy_ctx(ctx); }

const char* cofem_last_error(const cofem_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_err.c_str();
}

const char* cofem_status_string(cofem_status s) {
  switch (s) {
    case COFEM_OK: return "COFEM_OK";
    case COFEM_ERR_INVALID_ARG: return "COFEM_ERR_INVALID_ARG";
    case COFEM_ERR_OUT_OF_MEMORY: return "COFEM_ERR_OUT_OF_MEMORY";
    case COFEM_ERR_DEVICE: return "COFEM_ERR_DEVICE";
    case COFEM_ERR_NUMERIC: return "COFEM_ERR_NUMERIC";
    case COFEM_ERR_UNSUPPORTED: return "COFEM_ERR_UNSUPPORTED";
  }
  return "COFEM_UNKNOWN_STATUS";
}

}  // extern "C"

namespace {

cofem_status predictor_hook(cofem_ctx* c, void* user, float* d0, double* mu0) {
  return net_predict(static_cast<cofem_net*>(user), c->alpha, c->alpha_prev, c->xm, c->sdiag, c->taps,
                     c->cd.ks * c->cd.ks, c->beta, d0, mu0, c->stream);
}

}  // namespace

namespace cofem {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace cofem
