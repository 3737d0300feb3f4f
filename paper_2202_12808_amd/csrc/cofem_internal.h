// Internal declarations shared by the HIP translation units of libcofem.so.
//
// Device-side CG state.  Columns are numbered 0..KP-1 for probe slots
// (slots >= K hold zeros and stay zero) and KP for the mean column
// (beta Phi^T y, Eq. 7).  Probe columns are float32; the mean column is kept in
// float64 end to end, because its error is amplified by the conditioning of A
// (its right-hand side lies in the large-eigenvalue subspace of A while
// float32 rounding leaks into the alpha-sized directions).
#pragma once

#include <hip/hip_runtime.h>
#include "cofem.h"

#include <string>
#include <stddef.h>
#include <stdint.h>

namespace cofem {

constexpr int kMaxCols = 64;     // KP + 1 <= kMaxCols
constexpr int kThreads = 256;    // every kernel uses 256-thread blocks (4 wave64)
constexpr int kWaves = 4;
constexpr int kDenseKP = 32;     // dense probe block width (two 16-column MFMA blocks)

struct CgScalars {
  double rho[kMaxCols];   // ||r_c||^2 of the current residual
  double gam[kMaxCols];   // p_c^T A p_c
  double del[kMaxCols];   // r_c^T A p_c
  double eta[kMaxCols];   // ||A p_c||^2
  double a[kMaxCols];     // step lengths
  double b[kMaxCols];     // direction-update coefficients
  double nB;              // ||B||_F
  double ratio;           // sqrt(sum rho) / nB
  double tol;
  int32_t iter;           // CG iterations done in this solve
  int32_t stop;           // 1 once the solve is finished (kernels then no-op)
  int32_t limit;          // iteration cap
  int32_t fixed;          // 1: ignore tol, run exactly `limit` iterations
  int32_t kp;             // probe slots; index of the first mean column
  int32_t k;              // real probes
  int32_t nt;             // mean columns (tasks sharing alpha; 1 for one task)
  int32_t n_clamped;      // M-step floor hits of the last M-step
  int32_t numeric_error;  // set when a CG scalar is not finite
  uint32_t counter[4];    // last-block tickets (self-resetting)
  double true_res[kMaxCols];  // ||b_c - A x_c||^2 of the last solve (float64 sums)
  double true_ratio;          // sqrt(sum_c true_res[c]) / nB0
  double nB0;                 // ||B||_F of the E-step (nB is the current solve's reference)
  // per-column stop rule (COFEM_STOP_PER_COLUMN): column c is finished once
  // ||r_c|| < tol ||b_c|| and takes no further step; the solve stops when every
  // column is finished (or at the cap)
  int32_t per_col;            // 1: per-column rule, 0: joint Frobenius ratio
  int32_t all_done;           // per-column rule: every column finished
  int32_t done[kMaxCols];
  double bb[kMaxCols];        // ||b_c||^2 of the solve's right-hand side
  double gamma_change;        // M-step: ||1/alpha_new - 1/alpha_old|| / ||1/alpha_new||
};

// ---------------------------------------------------------------- device helpers
// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// Dictionary element i as stored by the caller: kind 0 float32, 1 float32 to
// be rounded to bfloat16 (the bfloat16 value is the problem), 2 bfloat16 bits.
enum { kDictF32 = 0, kDictF32ToBf16 = 1, kDictBf16 = 2 };
__device__ __forceinline__ uint32_t dict_bf16_bits(const void* phi, int kind, int64_t i) {
  if (kind == kDictBf16) return static_cast<const uint16_t*>(phi)[i];
  return bf16_rne_bits(static_cast<const float*>(phi)[i]);
}
__device__ __forceinline__ float dict_value(const void* phi, int kind, int64_t i) {
  if (kind == kDictF32) return static_cast<const float*>(phi)[i];
  return __uint_as_float(dict_bf16_bits(phi, kind, i) << 16);
}

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Rademacher sign of probe k, coordinate j, EM iteration t: bit (j & 63) of
// SplitMix64 output number (t<<48 | k<<32 | j>>6) + 1 for `seed`; 0 -> +1.
__device__ __forceinline__ float probe_sign(uint64_t seed, uint32_t t, uint32_t k, uint64_t j) {
  const uint64_t idx = ((uint64_t)t << 48) | ((uint64_t)k << 32) | (j >> 6);
  const uint64_t w = splitmix64_mix(seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
  return ((w >> (j & 63)) & 1ull) ? -1.0f : 1.0f;
}

// ||h||^2 in float64, the taps summed in order (every column of the
// convolution dictionary has this norm); loads go out in batches of 9 so a
// thread does not wait on each tap in turn.
__device__ __forceinline__ double taps_sq_sum(const float* __restrict__ taps, int ntaps) {
  double hh = 0.0;
  int i = 0;
  for (; i + 9 <= ntaps; i += 9) {
    float tv[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) tv[u] = taps[i + u];
#pragma unroll
    for (int u = 0; u < 9; ++u) hh += (double)tv[u] * (double)tv[u];
  }
  for (; i < ntaps; ++i) hh += (double)taps[i] * (double)taps[i];
  return hh;
}

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide "am I the last block to finish" ticket on `counter` (which the
// caller's last block resets to zero).  Every value another block will read
// must have been written with store_agent (an agent-coherent write-through
// store) and is read back with load_agent (an agent-coherent load).  Each
// thread waits for its own stores to complete before the barrier, so the
// ticket increment is ordered after all of the block's partials without a
// device-wide cache write-back per block.
// Ticket counters are spaced one 256-byte line apart (kCounterStride uint32
// slots): device-scope atomics on counters that share a line serialise at the
// memory side, and a reduction's level-one counters are hit by up to 32
// workgroups at once.  Arrays of counters are allocated and indexed with this
// stride.
constexpr int kCounterStride = 64;

__device__ __forceinline__ bool last_block_ticket(uint32_t* counter, uint32_t total) {
  __shared__ bool s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == total - 1u);
  }
  __syncthreads();
  return s_last;
}

// Sum of v over the block (blockDim.x a multiple of 64, at most 512 threads);
// result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* sh /* >= 8 doubles */) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) r += sh[w];
  return r;
}

// Deterministic tree reduction of per-block partial vectors across a grid.
// Every block calls it with its own ncols values in shared memory (`mine`,
// ncols <= blockDim.x); blocks are grouped 32 at a time per level, and the last
// block of each group sums the group (in index order) and moves up a level.
// Returns true in the single block that ends with the totals in `out_sh`.
// `parts` holds tree_rows(nblk) rows of ncols doubles and `cnts`
// tree_counters(nblk) zero-initialised counters, kCounterStride slots apart
// (left zero on exit).
__host__ __device__ __forceinline__ int64_t tree_rows(int64_t n) {
  int64_t rows = n;
  while (n > 1) {
    n = (n + 31) / 32;
    rows += n;
  }
  return rows;
}
__host__ __device__ __forceinline__ int64_t tree_counters(int64_t n) {
  int64_t c = 0;
  while (n > 1) {
    n = (n + 31) / 32;
    c += n;
  }
  return c < 1 ? 1 : c;
}

__device__ __forceinline__ bool tree_reduce(double* parts, uint32_t* cnts, int64_t blk, int64_t nblk,
                                            int ncols, const double* mine, double* out_sh) {
  const int tid = threadIdx.x;
  if (nblk == 1) {
    if (tid < ncols) out_sh[tid] = mine[tid];
    __syncthreads();
    return true;
  }
  if (tid < ncols) store_agent(&parts[blk * ncols + tid], mine[tid]);
  int64_t idx = blk, n = nblk;
  double* p = parts;
  uint32_t* c = cnts;
  for (;;) {
    const int64_t g = idx / 32;
    const int64_t base = g * 32;
    const int gs = (int)((n - base) < 32 ? (n - base) : 32);
    if (!last_block_ticket(&c[g * kCounterStride], (uint32_t)gs)) return false;
    double v = 0.0;
    if (tid < ncols) {
      // all (up to 32) loads in flight at once, summed in block order
      double t[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) t[u] = load_agent(&p[(base + (u < gs ? u : 0)) * ncols + tid]);
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (u < gs) v += t[u];
    }
    if (tid == 0) store_agent(&c[g * kCounterStride], 0u);
    const int64_t ng = (n + 31) / 32;
    if (ng == 1) {
      if (tid < ncols) out_sh[tid] = v;
      __syncthreads();
      return true;
    }
    double* pn = p + n * ncols;
    if (tid < ncols) store_agent(&pn[g * ncols + tid], v);
    c += ng * kCounterStride;
    p = pn;
    idx = g;
    n = ng;
  }
}

// Column-wise variant for grids of (block, column) pairs: block `blk` of
// column `col` holds nv values (`mine`).  Each column's blocks are summed by
// their own tree (parts/cnts regions of tree_rows(nblk)*nv doubles and
// tree_counters(nblk) counters per column); the block finishing a column
// stores the column's nv totals in colsum and takes a ticket on cnt_cols.
// The last of those returns true with every total in out_sh[v * ncols + col].
__device__ __forceinline__ bool column_tree_reduce(double* parts, uint32_t* cnts, double* colsum,
                                                   uint32_t* cnt_cols, int64_t blk, int64_t nblk,
                                                   int64_t nblk_alloc, int col, int ncols, int nv,
                                                   const double* mine, double* out_sh) {
  __shared__ double coltot[8];
  double* p = parts + (int64_t)col * tree_rows(nblk_alloc) * nv;
  uint32_t* c = cnts + (int64_t)col * tree_counters(nblk_alloc) * kCounterStride;
  if (!tree_reduce(p, c, blk, nblk, nv, mine, coltot)) return false;
  if (threadIdx.x < nv) store_agent(&colsum[col * nv + threadIdx.x], coltot[threadIdx.x]);
  if (!last_block_ticket(cnt_cols, (uint32_t)ncols)) return false;
  for (int e = threadIdx.x; e < ncols * nv; e += blockDim.x) {
    const int cc = e / nv, v = e - (e / nv) * nv;
    out_sh[v * ncols + cc] = load_agent(&colsum[e]);
  }
  if (threadIdx.x == 0) store_agent(cnt_cols, 0u);
  __syncthreads();
  return true;
}
__device__ __forceinline__ bool column_tree_reduce(double* parts, uint32_t* cnts, double* colsum,
                                                   uint32_t* cnt_cols, int64_t blk, int64_t nblk,
                                                   int col, int ncols, int nv, const double* mine,
                                                   double* out_sh) {
  return column_tree_reduce(parts, cnts, colsum, cnt_cols, blk, nblk, nblk, col, ncols, nv, mine, out_sh);
}

// ------------------------------------------------ per-block column sums (dense)
// Thread tid owns probe column tid & 31 (acc) and a share of each of the nt
// mean columns (accm[j]); leaves the block's kDenseKP + nt sums in out_sh
// (256-thread blocks).
constexpr int kMaxDenseTasks = 4;  // mean columns of a dense problem (tasks sharing alpha)

__device__ __forceinline__ void dense_block_sums(double acc, const double* accm, int nt, double* out_sh) {
  __shared__ double sh[kThreads];
  __shared__ double shm[8];
  __shared__ double msum[kMaxDenseTasks];
  sh[threadIdx.x] = acc;
  for (int j = 0; j < nt; ++j) {
    const double m = block_sum(accm[j], shm);  // synchronises
    if (threadIdx.x == 0) msum[j] = m;
  }
  __syncthreads();
  if (threadIdx.x < kDenseKP) {
    double v = 0.0;
    for (int t = threadIdx.x; t < kThreads; t += kDenseKP) v += sh[t];
    out_sh[threadIdx.x] = v;
  } else if (threadIdx.x < kDenseKP + nt) {
    out_sh[threadIdx.x] = msum[threadIdx.x - kDenseKP];
  }
  __syncthreads();
}
__device__ __forceinline__ void dense_block_sums(double acc, double accm, double* out_sh) {
  dense_block_sums(acc, &accm, 1, out_sh);
}

// The finish_* helpers run in the last block of a reduction, all threads,
// with the per-column totals in shared memory.  Column c is handled by thread
// c, so the loads of the scalar block are issued together (one round trip to
// device-coherent memory, not one per column); column sums are formed by
// thread 0 from shared memory in column order.

// The scalars that the finishing block of a CG kernel reads, loaded by every
// block at kernel start (they do not change during the kernel), so the last
// block's finish costs no further memory round trip.
struct CgCtl {
  double rho;  // st->rho[threadIdx.x] in threads < nc, else 0
  double bb;   // per-column rule: st->bb[threadIdx.x] in threads < nc
  double nB, tol;
  int nc, iter, limit, fixed;
  int per_col, done;  // done: st->done[threadIdx.x] (per-column rule)
};
__device__ __forceinline__ CgCtl load_cg_ctl(const CgScalars* st) {
  CgCtl c;
  c.nc = st->kp + st->nt;
  const bool mine = (int)threadIdx.x < c.nc;
  c.rho = mine ? st->rho[threadIdx.x] : 0.0;
  c.nB = st->nB;
  c.tol = st->tol;
  c.iter = st->iter;
  c.limit = st->limit;
  c.fixed = st->fixed;
  c.per_col = st->per_col;
  c.done = (c.per_col && mine) ? st->done[threadIdx.x] : 0;
  c.bb = (c.per_col && mine) ? st->bb[threadIdx.x] : 0.0;
  return c;
}

// Per-column stop rule: thread c < nc decides whether its column is finished
// after a residual norm ||r_c||^2 = rr (sticky: a finished column stays
// finished), stores the flag, and the block learns whether all are finished.
// Every thread of the block must call it.  Without the rule it returns false.
__device__ __forceinline__ bool per_column_finish(CgScalars* st, const CgCtl& k, double rr, int* done_out) {
  __shared__ int s_open;
  if (!k.per_col) {
    *done_out = 0;
    return false;
  }
  if (threadIdx.x == 0) s_open = 0;
  __syncthreads();
  const int c = threadIdx.x;
  int d = 0;
  if (c < k.nc) {
    d = k.done || (!k.fixed && (k.bb == 0.0 || sqrt(rr) < k.tol * sqrt(k.bb)));
    st->done[c] = d;
    if (!d) atomicAdd(&s_open, 1);
  }
  __syncthreads();
  *done_out = d;
  return s_open == 0;
}

// Finishes a CG update: the new ||r_c||^2 for columns 0..kp.  Applies the stop
// test of the solve (joint Frobenius ratio of the recursive residual, or the
// cap).
__device__ __forceinline__ void finish_update(CgScalars* st, const double* new_rho, const CgCtl& k) {
  const int nc = k.nc;
  if ((int)threadIdx.x < nc) st->rho[threadIdx.x] = new_rho[threadIdx.x];
  int mine_done;
  const bool all = per_column_finish(st, k, (int)threadIdx.x < nc ? new_rho[threadIdx.x] : 0.0, &mine_done);
  if (threadIdx.x == 0) {
    const int it = k.iter + 1;
    double sum = 0.0;
    for (int c = 0; c < nc; ++c) sum += new_rho[c];
    const bool finite = isfinite(sum);
    if (!finite) st->numeric_error = 1;
    const double ratio = k.nB > 0.0 ? sqrt(sum) / k.nB : 0.0;
    st->ratio = ratio;
    st->iter = it;
    st->all_done = all ? 1 : 0;
    const bool met = k.per_col ? all : (!k.fixed && ratio < k.tol);
    st->stop = (it >= k.limit) || met || !finite;
  }
}
__device__ __forceinline__ void finish_update(CgScalars* st, const double* new_rho) {
  finish_update(st, new_rho, load_cg_ctl(st));
}

// Finishes a preconditioned CG update (z = M^-1 r): v holds, per column (nc
// values each), rho' = r^T z and r^T r.  rho <- rho' (the next step length's
// numerator), the iteration count, and the stop test on the unpreconditioned
// residual, sqrt(sum r^T r) / ||B||_F (Sec. 3.2), or the per-column rule on
// r^T r.
__device__ __forceinline__ void finish_update_pcg(CgScalars* st, const double* v, int nc, const CgCtl& k) {
  if ((int)threadIdx.x < nc) st->rho[threadIdx.x] = v[threadIdx.x];
  int mine_done;
  const bool all = per_column_finish(st, k, (int)threadIdx.x < nc ? v[nc + threadIdx.x] : 0.0, &mine_done);
  if (threadIdx.x == 0) {
    const int it = k.iter + 1;
    double rr = 0.0, rz = 0.0;
    for (int c = 0; c < nc; ++c) {
      rz += v[c];
      rr += v[nc + c];
    }
    const bool finite = isfinite(rr) && isfinite(rz);
    if (!finite) st->numeric_error = 1;
    const double ratio = k.nB > 0.0 ? sqrt(rr) / k.nB : 0.0;
    st->ratio = ratio;
    st->iter = it;
    st->all_done = all ? 1 : 0;
    const bool met = k.per_col ? all : (!k.fixed && ratio < k.tol);
    st->stop = (it >= k.limit) || met || !finite;
  }
}

// Finishes a step-length computation from the three dot products of the
// operator pass (gam = p^T q, del = r^T q, eta = q^T q, each kp+1 entries in
// shared memory, laid out gam | del | eta):
//   a_c = rho_c / gam_c, and the direction-update coefficient
//   b_c = ||r_c - a_c q_c||^2 / rho_c = (rho_c - 2 a_c del_c + a_c^2 eta_c) / rho_c
// (the same value Hestenes-Stiefel CG forms after the residual update; known
// here one kernel earlier so the update kernel can also form p <- r + b p).
__device__ __forceinline__ void finish_step(CgScalars* st, const double* dots, const CgCtl& k) {
  __shared__ int s_bad;
  const int nc = k.nc;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const int c = threadIdx.x;
  if (c < nc) {
    const double g = dots[c], dl = dots[nc + c], et = dots[2 * nc + c];
    const double rho = k.rho;
    // a finished column (per-column rule) takes no step
    const double a = (g != 0.0 && !k.done) ? rho / g : 0.0;
    st->gam[c] = g;
    st->del[c] = dl;
    st->eta[c] = et;
    st->a[c] = a;
    double rn = rho - 2.0 * a * dl + a * a * et;
    if (rn < 0.0) rn = 0.0;
    st->b[c] = (rho != 0.0 && !k.done) ? rn / rho : 0.0;
    if (!(isfinite(g) && isfinite(dl) && isfinite(et))) s_bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_bad) {
    st->numeric_error = 1;
    st->stop = 1;
  }
}
__device__ __forceinline__ void finish_step(CgScalars* st, const double* dots) {
  finish_step(st, dots, load_cg_ctl(st));
}

// Finishes a fused conv iteration (an update followed by an operator pass):
// v holds, per column (nc values each), rho' = r^T z, r^T r, gam, del, eta.
// The update's part: rho <- rho', the iteration count and the stop test on
// sqrt(sum r^T r) / ||B||_F (as finish_update_pcg); then, for the next
// update, a = rho'/gam and b = (rho' - 2 a del + a^2 eta)/rho' (as
// finish_step).
__device__ __forceinline__ void finish_fused(CgScalars* st, const double* v, int nc, const CgCtl& k) {
  __shared__ int s_bad;
  int mine_done;
  const bool all = per_column_finish(st, k, (int)threadIdx.x < nc ? v[nc + threadIdx.x] : 0.0, &mine_done);
  if (threadIdx.x == 0) {
    const int it = k.iter + 1;
    double rr = 0.0, rz = 0.0;
    for (int c = 0; c < nc; ++c) {
      rz += v[c];
      rr += v[nc + c];
    }
    const bool finite = isfinite(rr) && isfinite(rz);
    const double ratio = k.nB > 0.0 ? sqrt(rr) / k.nB : 0.0;
    st->ratio = ratio;
    st->iter = it;
    st->all_done = all ? 1 : 0;
    s_bad = finite ? 0 : 1;
    const bool met = k.per_col ? all : (!k.fixed && ratio < k.tol);
    st->stop = (it >= k.limit) || met || !finite;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < nc) {
    const double rho = v[c], g = v[2 * nc + c], dl = v[3 * nc + c], et = v[4 * nc + c];
    st->rho[c] = rho;
    // a finished column (per-column rule) takes no further step
    const double a = (g != 0.0 && !mine_done) ? rho / g : 0.0;
    st->gam[c] = g;
    st->del[c] = dl;
    st->eta[c] = et;
    st->a[c] = a;
    double rn = rho - 2.0 * a * dl + a * a * et;
    if (rn < 0.0) rn = 0.0;
    st->b[c] = (rho != 0.0 && !mine_done) ? rn / rho : 0.0;
    if (!(isfinite(g) && isfinite(dl) && isfinite(et))) s_bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_bad) {
    st->numeric_error = 1;
    st->stop = 1;
  }
}

// Finishes the initial residual R = B: rho_c = ||b_c||^2 (in shared memory).
// Start-of-solve part of the per-column rule: thread c < nc records
// ||b_c||^2 = bb and whether the column is finished already (||r_c||^2 = rr
// at the start; a zero right-hand side is finished).  Returns (to every
// thread) whether all columns are.
__device__ __forceinline__ bool per_column_start(CgScalars* st, int nc, double rr, double bb) {
  __shared__ int s_open;
  const int per_col = st->per_col, fixed = st->fixed;
  const double tol = st->tol;
  if (threadIdx.x == 0) s_open = 0;
  __syncthreads();
  const int c = threadIdx.x;
  if (c < nc) {
    const int d = per_col && !fixed && (bb == 0.0 || sqrt(rr) < tol * sqrt(bb));
    st->done[c] = d;
    st->bb[c] = bb;
    if (!d) atomicAdd(&s_open, 1);
  }
  __syncthreads();
  return per_col && s_open == 0;
}

__device__ __forceinline__ void finish_init(CgScalars* st, const double* rho) {
  const int nc = st->kp + st->nt;
  if ((int)threadIdx.x < nc) {
    st->rho[threadIdx.x] = rho[threadIdx.x];
    st->b[threadIdx.x] = 0.0;
    st->a[threadIdx.x] = 0.0;
  }
  const double own = (int)threadIdx.x < nc ? rho[threadIdx.x] : 0.0;
  const bool all = per_column_start(st, nc, own, own);
  if (threadIdx.x == 0) {
    const int limit = st->limit, fixed = st->fixed;
    const double tol = st->tol;
    double sum = 0.0;
    for (int c = 0; c < nc; ++c) sum += rho[c];
    st->nB = sqrt(sum);
    st->nB0 = sqrt(sum);
    st->ratio = sum > 0.0 ? 1.0 : 0.0;
    st->iter = 0;
    st->n_clamped = 0;
    st->all_done = all ? 1 : 0;
    st->numeric_error = isfinite(sum) ? 0 : 1;
    const bool met = st->per_col ? all : (!fixed && 1.0 < tol);
    st->stop = (sum == 0.0) || (limit <= 0) || met || !isfinite(sum);
  }
}

// Finishes the start of a preconditioned solve: per column r^T z, ||r||^2 and
// ||b||^2 in shared memory (laid out value-major, ncols each).
__device__ __forceinline__ void finish_init_pcg(CgScalars* st, const double* v, int ncols) {
  if ((int)threadIdx.x < ncols) {
    st->rho[threadIdx.x] = v[threadIdx.x];
    st->a[threadIdx.x] = 0.0;
    st->b[threadIdx.x] = 0.0;
  }
  const bool mine = (int)threadIdx.x < ncols;
  const bool all = per_column_start(st, ncols, mine ? v[ncols + threadIdx.x] : 0.0,
                                    mine ? v[2 * ncols + threadIdx.x] : 0.0);
  if (threadIdx.x == 0) {
    const int limit = st->limit, fixed = st->fixed;
    const double tol = st->tol;
    double rr = 0.0, bb = 0.0, rz = 0.0;
    for (int c = 0; c < ncols; ++c) {
      rz += v[c];
      rr += v[ncols + c];
      bb += v[2 * ncols + c];
    }
    const bool finite = isfinite(rz) && isfinite(rr) && isfinite(bb);
    const double nB = sqrt(bb);
    st->nB = nB;
    st->nB0 = nB;
    st->ratio = nB > 0.0 ? sqrt(rr) / nB : 0.0;
    st->iter = 0;
    st->n_clamped = 0;
    st->all_done = all ? 1 : 0;
    st->numeric_error = finite ? 0 : 1;
    const bool met = st->per_col ? all : (!fixed && st->ratio < tol);
    st->stop = (bb == 0.0) || (limit <= 0) || met || !finite;
  }
}

// Finishes the M-step's sums (in shared memory: floor hits, the squared
// change of the prior variances 1/alpha, their squared norm): the clamp count
// and the relative change ||1/alpha_new - 1/alpha_old|| / ||1/alpha_new||.
__device__ __forceinline__ void finish_mstep(CgScalars* st, const double* v) {
  if (threadIdx.x == 0) {
    st->n_clamped = (int32_t)v[0];
    st->gamma_change = v[2] > 0.0 ? sqrt(v[1]) / sqrt(v[2]) : 0.0;
  }
}

// Finishes the true-residual check: ||b_c - A x_c||^2 per column (in shared
// memory) and the joint ratio sqrt(sum_c ...) / ||B||_F.
__device__ __forceinline__ void finish_true_resid(CgScalars* st, const double* res) {
  const int nc = st->kp + st->nt;
  if ((int)threadIdx.x < nc) st->true_res[threadIdx.x] = res[threadIdx.x];
  if (threadIdx.x == 0) {
    const double nB = st->nB;
    double sum = 0.0;
    for (int c = 0; c < nc; ++c) sum += res[c];
    if (!isfinite(sum)) st->numeric_error = 1;
    st->true_ratio = nB > 0.0 ? sqrt(sum) / nB : 0.0;
  }
}

// Finishes the outer residual of an iterative-refinement sweep (||r_c||^2 in
// shared memory): the next inner solve starts from R with reference norm
// ||R||_F, a fresh iteration count and cap `limit`; true_ratio = ||R||_F/||B||_F.
__device__ __forceinline__ void finish_ir_residual(CgScalars* st, const double* rho, int limit) {
  const int nc = st->kp + st->nt;
  if ((int)threadIdx.x < nc) {
    st->rho[threadIdx.x] = rho[threadIdx.x];
    st->true_res[threadIdx.x] = rho[threadIdx.x];
    st->a[threadIdx.x] = 0.0;
    st->b[threadIdx.x] = 0.0;
  }
  if (threadIdx.x == 0) {
    const double nB0 = st->nB0;
    double sum = 0.0;
    for (int c = 0; c < nc; ++c) sum += rho[c];
    const bool finite = isfinite(sum);
    const double nr = sqrt(sum);
    st->nB = nr;
    st->true_ratio = nB0 > 0.0 ? nr / nB0 : 0.0;
    st->ratio = sum > 0.0 ? 1.0 : 0.0;
    st->iter = 0;
    st->limit = limit;
    if (!finite) st->numeric_error = 1;
    st->stop = (sum == 0.0) || (limit <= 0) || !finite;
  }
}

// The preconditioned form of finish_ir_residual: v holds, per column (nc
// values each), r^T z and r^T r of the new outer residual R and Z = M^-1 R.
// rho <- r^T z; the reference norm and the true ratio come from r^T r.
__device__ __forceinline__ void finish_ir_residual_pcg(CgScalars* st, const double* v, int limit) {
  const int nc = st->kp + st->nt;
  if ((int)threadIdx.x < nc) {
    st->rho[threadIdx.x] = v[threadIdx.x];
    st->true_res[threadIdx.x] = v[nc + threadIdx.x];
    st->a[threadIdx.x] = 0.0;
    st->b[threadIdx.x] = 0.0;
  }
  if (threadIdx.x == 0) {
    const double nB0 = st->nB0;
    double rr = 0.0, rz = 0.0;
    for (int c = 0; c < nc; ++c) {
      rz += v[c];
      rr += v[nc + c];
    }
    const bool finite = isfinite(rr) && isfinite(rz);
    const double nr = sqrt(rr);
    st->nB = nr;
    st->true_ratio = nB0 > 0.0 ? nr / nB0 : 0.0;
    st->ratio = rr > 0.0 ? 1.0 : 0.0;
    st->iter = 0;
    st->limit = limit;
    if (!finite) st->numeric_error = 1;
    st->stop = (rr == 0.0) || (limit <= 0) || !finite;
  }
}

// ------------------------------------------------------------ host launchers
// Dense problem geometry.  Np and Dp are N and D padded to multiples of 64.
// Probe-column state uses the blocked-4 layout: element (d, c) of a Dp x 32
// block lives at (d / 4) * 128 + c * 4 + d % 4, so four consecutive
// coordinates of one column form a float4 (the MFMA B-operand and C-result
// shape of v_mfma_f32_16x16x4f32).
struct DenseDims {
  int64_t N, D, Np, Dp;
  int S1, S2;  // workgroups sharing one tile's reduction in pass 1 / pass 2
  int ring;    // outstanding 8-wide groups per wave (1, 2, 4 or 8)
  int S1h, S2h;  // splits of the bfloat16 passes (two tiles per workgroup)
  int nt = 1;    // float64 mean columns (tasks sharing alpha), stride Dp (Np for W)
};

__host__ __device__ __forceinline__ int64_t blk4(int64_t d, int c) {
  return (d >> 2) * 128 + c * 4 + (d & 3);
}

hipError_t dense_pack(const float* phi, int64_t ld, const DenseDims& dd, float* phiA, float* phiB,
                      hipStream_t s);
hipError_t dense_b0(const void* phi, int dict_kind, int64_t ld, const float* y, double beta, const DenseDims& dd,
                    double* b0, hipStream_t s);
// minv (dense vector kernels and the second passes): the Jacobi diagonal
// M^-1 (Dp floats, zero in the padding rows), or null for plain CG.  With it
// the start and the update form z = M^-1 r, p = z + b p, r^T z (the step's
// numerator) and r^T r (the stop test); the second pass weights its del and
// eta by M^-1.
hipError_t dense_init(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0,
                      float* X, float* R, float* P, double* xm, double* rm, double* pm,
                      double* parts, uint32_t* cnts, CgScalars* st, hipStream_t s, const float* minv = nullptr);
hipError_t dense_pass1(const DenseDims& dd, const float* phiA, const float* P, const double* pm,
                       float* Wpart, double* wmpart, float* W, double* wm, uint32_t* cnts,
                       CgScalars* st, int apply_only, hipStream_t s);
hipError_t dense_pass2(const DenseDims& dd, const float* phiB, const float* W, const double* wm,
                       const float* P, const double* pm, const float* R, const double* rm,
                       const float* alpha, double beta, float* Qpart, double* qmpart, float* Q,
                       double* qm, double* gpart, uint32_t* counter, uint32_t* split_cnts,
                       CgScalars* st, int apply_only, hipStream_t s, const float* minv = nullptr);
hipError_t dense_update(const DenseDims& dd, float* X, float* R, float* P, const float* Q,
                        double* xm, double* rm, double* pm, const double* qm, double* parts,
                        uint32_t* cnts, CgScalars* st, hipStream_t s, const float* minv = nullptr);
// ||Phi e_d||^2 for d < D (float64 sums over the caller's Phi), zero in the padding
hipError_t dense_colnorms(const void* phi, int dict_kind, int64_t ld, const DenseDims& dd, float* cn,
                          hipStream_t s);
// M^-1 = 1 / (beta ||Phi e_d||^2 + alpha_d) for d < D, zero in the padding
hipError_t dense_jacobi(const DenseDims& dd, const float* cn, double beta, const float* alpha, float* minv,
                        hipStream_t s);
int dense_split(int64_t tiles, int64_t groups, int nt = 1);
bool dense_split_ok(int64_t groups, int splits, int nt = 1);
// diagonal estimate and M-step; the update's reduction tree (parts, cnts)
// serves its sums (clamp count, change of 1/alpha)
hipError_t dense_mstep(const DenseDims& dd, uint64_t seed, int t, int K, const float* X,
                       const double* xm, float* alpha, double alpha_max, float* mu, float* sdiag,
                       double* parts, uint32_t* cnts, CgScalars* st, hipStream_t s);
hipError_t dense_to_colmajor(const DenseDims& dd, int K, const float* Xb, float* out, hipStream_t s);
hipError_t dense_from_colmajor(const DenseDims& dd, int K, const float* in, float* Xb, hipStream_t s);
int dense_update_blocks(const DenseDims& dd);
// bfloat16-dictionary passes of the mixed-precision form (kernels_dense_bf16.hip)
hipError_t dense_pack16(const void* phi, int dict_kind, int64_t ld, const DenseDims& dd, void* phiA16,
                        void* phiB16, hipStream_t s);
int dense16_split(int64_t pairs, int64_t groups);
bool dense16_split_ok(int64_t groups, int splits);
hipError_t dense16_pass1(const DenseDims& dd, const void* phiA16, const float* P, const double* pm,
                         float* Wpart, double* wmpart, float* W, double* wm, uint32_t* cnts, CgScalars* st,
                         int apply_only, hipStream_t s);
hipError_t dense16_pass2(const DenseDims& dd, const void* phiB16, const float* W, const double* wm,
                         const float* P, const double* pm, const float* R, const double* rm, const float* alpha,
                         double beta, float* Qpart, double* qmpart, float* Q, double* qm, double* gpart,
                         uint32_t* counter, uint32_t* split_cnts, CgScalars* st, int apply_only, hipStream_t s,
                         const float* minv = nullptr);
// Xt's probe columns <- max(s_prev, 0) (.) p_k (EM iteration t); the mean column is kept
hipError_t dense_warm_start(const DenseDims& dd, uint64_t seed, int t, int K, const float* sprev, float* Xt,
                            hipStream_t s);
hipError_t dense_ir_accumulate(const DenseDims& dd, float* Xt, const float* Xi, double* xtm, const double* xim,
                               hipStream_t s);
hipError_t dense_ir_residual(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0, const float* Q,
                             const double* qm, float* Xi, float* R, float* P, double* xim, double* rm, double* pm,
                             double* parts, uint32_t* cnts, CgScalars* st, int limit, hipStream_t s,
                             const float* minv = nullptr);
// ||B - Q||^2 per column with B regenerated (probes of EM iteration t, b0) and
// Q = A X from the operator passes (blocked-4 probe block + float64 column).
hipError_t dense_true_resid(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0,
                            const float* Q, const double* qm, double* parts, uint32_t* cnts,
                            CgScalars* st, hipStream_t s);

constexpr int kConvTile = 64;  // output tile side of the fused conv operator pass

struct ConvDims {
  int H, W, ks;      // square odd kernel side
  int64_t D, ldD;    // D = H*W, ldD = D rounded up to 256
  int K;             // probe columns (column-major blocks of ldD elements)
  int tilesX, tilesY;  // kConvTile x kConvTile output tiles
  int fp64;          // probe columns in float64 (else float32)
  // element order of the state vectors: 0 = natural; otherwise l1 | (l2 << 8)
  // for the DCT dictionary's row-major order of coefficient k = k1 + 2^l1 k2
  // at position k1 2^l2 + k2 (perm_nat maps a position to k)
  int perm;
  // float64 mean columns (tasks sharing alpha), blocks of ldD after xm etc.
  int nt;
  // workgroups of the persistent warp-specialised fused iteration
  // (kernels_conv_ws.hip); 0: the per-tile kernel
  int ws_grid;
};

__host__ __device__ __forceinline__ int64_t perm_nat(int perm, int64_t pos) {
  if (perm == 0) return pos;
  const int l1 = perm & 0xFF, l2 = perm >> 8;
  return (pos >> l2) + ((pos & ((int64_t(1) << l2) - 1)) << l1);
}

hipError_t conv_b0(const ConvDims& cd, const float* taps, const float* y, double beta, double* b0,
                   hipStream_t s);
// Reduction workspace of the conv kernels (one region per column).
struct ConvReduce {
  double* parts;      // (K+1) regions of tree_rows(nblk) * nv doubles
  uint32_t* cnts;     // (K+1) regions of tree_counters(nblk)
  double* colsum;     // (K+1) * 3 doubles
  uint32_t* cnt_cols; // 1 counter
};

// Probe-column blocks are float or double according to cd.fp64.
hipError_t conv_init(const ConvDims& cd, uint64_t seed, int t, const double* b0, void* X, void* R,
                     void* P, double* xm, double* rm, double* pm, const ConvReduce& red,
                     CgScalars* st, hipStream_t s);
int64_t conv_pass_blocks(const ConvDims& cd);
// One of the two buffer sets of the conv CG direction, residual and operator
// product (probe columns of the context's type, mean column float64).
struct ConvState {
  void *P, *R, *Q;
  double *pm, *rm, *qm;
};
hipError_t conv_fused(const ConvDims& cd, const float* taps, const ConvState& s0, const ConvState& s1, void* X,
                      double* xm, const float* alpha, double beta, const float* minv, const ConvReduce& red,
                      CgScalars* st, hipStream_t s);
// The persistent warp-specialised forms of conv_fused and conv_pass (float
// probe columns): whether the problem's shape admits them, and the launches
// on `grid` workgroups.
bool conv_ws_ok(const ConvDims& cd);
hipError_t conv_fused_ws(const ConvDims& cd, int grid, const float* taps, const ConvState& s0, const ConvState& s1,
                         void* X, double* xm, const float* alpha, double beta, const float* minv,
                         const ConvReduce& red, CgScalars* st, hipStream_t s);
hipError_t conv_pass_ws(const ConvDims& cd, int grid, const float* taps, const void* P, const double* pm,
                        const void* R, const double* rm, const float* alpha, double beta, void* Q, double* qm,
                        const ConvReduce& red, CgScalars* st, int apply_only, hipStream_t s, const float* minv);
// The start of a warm-started solve (conv_init_pcg on A X0, with A X0 formed
// in the same launch) and the true-residual check (conv_true_resid on A X),
// as modes of the persistent kernel; natural element order.
hipError_t conv_init_ws(const ConvDims& cd, int grid, const float* taps, uint64_t seed, int t, const double* b0,
                        const float* minv, const void* X, const double* xm, void* R, void* P, double* rm,
                        double* pm, const float* alpha, double beta, const ConvReduce& red, CgScalars* st,
                        hipStream_t s);
// only_if_stopped: the launch does nothing unless the solve's stop flag is set
// when it starts (a residual enqueued before the host has read the flag)
hipError_t conv_resid_ws(const ConvDims& cd, int grid, const float* taps, uint64_t seed, int t, const double* b0,
                         const void* X, const double* xm, const float* alpha, double beta, const ConvReduce& red,
                         CgScalars* st, hipStream_t s, bool only_if_stopped = false);
hipError_t conv_pass(const ConvDims& cd, const float* taps, const void* P, const double* pm,
                     const void* R, const double* rm, const float* alpha, double beta, void* Q,
                     double* qm, const ConvReduce& red, CgScalars* st, int apply_only, hipStream_t s,
                     const float* minv = nullptr);
// preconditioned CG from a starting block (warm-started and learned forms)
hipError_t conv_init_pcg(const ConvDims& cd, uint64_t seed, int t, const double* b0, const float* minv,
                         const void* Qx, const double* qxm, void* X, void* R, void* P, double* xm, double* rm,
                         double* pm, const ConvReduce& red, CgScalars* st, hipStream_t s);
hipError_t conv_start(const ConvDims& cd, uint64_t seed, int t, const float* d0, const double* mu0, void* X,
                      double* xm, hipStream_t s);
hipError_t conv_jacobi(const ConvDims& cd, const float* taps, double beta, const float* alpha, float* minv,
                       hipStream_t s);
hipError_t conv_true_resid(const ConvDims& cd, uint64_t seed, int t, const double* b0, const void* Q,
                           const double* qm, const ConvReduce& red, CgScalars* st, hipStream_t s);
// alpha_prev (may be null): receives the alpha this M-step replaces
hipError_t conv_mstep(const ConvDims& cd, uint64_t seed, int t, const void* X, const double* xm,
                      float* alpha, double alpha_max, float* mu, float* sdiag, const ConvReduce& red, CgScalars* st,
                      hipStream_t s, float* alpha_prev = nullptr);
hipError_t conv_probes_out(const ConvDims& cd, const void* X, float* out, hipStream_t s);
hipError_t conv_probes_in(const ConvDims& cd, const float* in, void* X, hipStream_t s);

// Spectral start (kernels_spectral.hip): with a uniform alpha = a0, the start
// block X0 = A^-1 [p_1 .. p_K | b0_1 .. b0_T] by 2D DFTs, for power-of-two H
// and W up to kSpecMaxSide.  Tables: g (D floats, |h_hat|^2) and tw
// (conv_spectral_twiddles float2); workspace Z: conv_spectral_pairs * D float2.
constexpr int kSpecMaxSide = 4096;
bool conv_spectral_ok(int H, int W);
int64_t conv_spectral_pairs(const ConvDims& cd);
int64_t conv_spectral_twiddles(const ConvDims& cd);
hipError_t conv_spectral_tables(const ConvDims& cd, const float* taps, float* g, float2* tw, hipStream_t s);
hipError_t conv_spectral_start(const ConvDims& cd, uint64_t seed, int t, const double* b0, const float* g,
                               const float2* tw, double beta, double a0, float2* Z, void* X, double* xm,
                               hipStream_t s);

hipError_t probe_signs_colmajor(uint64_t seed, int t, int K, int64_t D, float* out, hipStream_t s);
hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t s);

int conv_update_blocks(const ConvDims& cd);
// element-order conversions of the state (cd.perm) to and from the caller's
// natural order: float vectors, float64 vectors
hipError_t perm_out_f32(const ConvDims& cd, const float* src, float* dst, hipStream_t s);
hipError_t perm_in_f32(const ConvDims& cd, const float* src, float* dst, hipStream_t s);
hipError_t perm_out_f64(const ConvDims& cd, const double* src, double* dst, hipStream_t s);
hipError_t perm_in_f64(const ConvDims& cd, const double* src, double* dst, hipStream_t s);

// ------------------------------------------------------------ DCT dictionary
// Phi = S C^T: the orthonormal inverse DCT of a length-D coefficient vector,
// then N observed samples.  A v = beta C S^T S C^T v + alpha v runs as one
// complex FFT sandwich per pair of float columns (and one for the float64
// mean column): D = N1 N2 in the four-step order, three launches per CG
// iteration: rows of the state (length-N2 transforms, with the previous CG
// update folded in), then groups of the intermediate (length-N1 inverse and
// forward transforms around the mask), then rows again (forward, the
// operator's output and the CG dot products).  State vectors are in the row
// order of ConvDims::perm.
struct DctDims {
  int64_t D;
  int l1, l2;      // N1 = 2^l1 rows, N2 = 2^l2 columns (l1 = ceil(p/2))
  int K;           // probe columns
  int npairs;      // ceil(K/2) float column pairs
  int nt, ntd;     // float64 mean columns (tasks) and their pairs ceil(nt/2)
  int units;       // N1/2 + 1 row units (a row and its mirror row)
  int gf, gd;      // groups per middle-launch tile: float pairs, float64 column
};
struct DctBuffers {
  float* Wf;             // npairs x D complex float intermediates
  double* Wd;            // ntd x D complex double intermediates (mean column pairs)
  const uint8_t* mk;     // mask: 1 where the sample is observed, middle-launch order
  double mval;           // the mask's scale beta/D
  const float* tw1f;     // e^{2 pi i j / N1}, j < N1 (float complex)
  const float* tw2f;     // e^{2 pi i j / N2}
  const double* tw1d;
  const double* tw2d;
  double* rr;            // per (column, row unit): r^T z, then (second half) r^T r of the folded update
};
// Set-up: mask bytes and the zero-filled scaled data for b0, twiddle tables,
// then b0 = beta Phi^T y (float64, state order) and, if cn is not null, the
// squared column norms ||Phi e_k||^2 (state order).  rows: device int32 [N].
hipError_t dct_setup(const DctDims& dd, const int32_t* rows, int64_t N, const float* y, double beta, uint8_t* mk,
                     double* vb, float* tw1f, float* tw2f, double* tw1d, double* tw2d, const DctBuffers& b,
                     double* b0, double* cn, hipStream_t s);
// Jacobi preconditioner minv = 1 / (beta cn + alpha), state order.
hipError_t dct_jacobi(const DctDims& dd, const double* cn, double beta, const float* alpha, float* minv,
                      hipStream_t s);
// One CG iteration is dct_rows_in, dct_mid, dct_rows_out.  fused = 0: Q = A P with the pass's
// dot products (first iteration of a solve); fused = 1: the previous update
// (x += a p, r -= a q, p = r + b p, in place) folded into the first launch,
// then Q = A P; apply_only: Q = A P with no reduction and no stop check.
// minv (null: none) preconditions the folded update: z = M^-1 r, p = z + b p.
hipError_t dct_rows_in(const DctDims& dd, const DctBuffers& b, void* X, void* R, void* P, const void* Q, double* xm,
                       double* rm, double* pm, const double* qm, const float* minv, CgScalars* st, int fused,
                       int apply_only, hipStream_t s);
hipError_t dct_mid(const DctDims& dd, const DctBuffers& b, CgScalars* st, int apply_only, hipStream_t s);
// minv (null: none) weights the pass's dots r^T M^-1 q and q^T M^-1 q.
hipError_t dct_rows_out(const DctDims& dd, const DctBuffers& b, const void* P, const void* R, void* Q,
                        const double* pm, const double* rm, double* qm, const float* alpha, const float* minv,
                        const ConvReduce& red, CgScalars* st, int fused, int apply_only, hipStream_t s);

// ------------------------------------------------------------ batched form
// Many independent dense problems (bfloat16 dictionaries, plain CG) advanced
// together: every grouped launch covers all problems' blocks, each block
// reading its (problem, a, b) work item and the problem's descriptor.
struct BatchProblem {
  int64_t N, D, Np, Dp;
  int32_t S1, S2;          // reduction splits of pass 1 / pass 2
  int32_t npairs1, npairs2;  // Np / 64, Dp / 64 (two tiles per workgroup)
  int32_t nvec;            // blocks of the vector kernels (init, update, M-step)
  int32_t pad;
  uint64_t seed;           // probe seed of this problem
  const void* phiA16;
  const void* phiB16;
  const double* b0;
  float* alpha;
  float *X, *R, *P, *Q, *W, *Wpart, *Qpart;
  double *xm, *rm, *pm, *qm, *wm, *wmpart, *qmpart;
  uint32_t *cnt_split1, *cnt_split2;
  double *parts_init, *parts_upd, *parts_pass;
  uint32_t *cnts_init, *cnts_upd, *cnts_pass;
  float *mu, *sdiag;
  CgScalars* st;
};
struct BatchItem {
  int32_t prob, a, b, pad;  // pass kernels: a = tile pair, b = split; vector kernels: a = block
};
hipError_t batch_pass1(const BatchItem* items, int n, const BatchProblem* probs, int apply_only, hipStream_t s);
hipError_t batch_pass2(const BatchItem* items, int n, const BatchProblem* probs, double beta, int apply_only,
                       hipStream_t s);
hipError_t batch_init(const BatchItem* items, int n, const BatchProblem* probs, int t, int K, hipStream_t s);
hipError_t batch_update(const BatchItem* items, int n, const BatchProblem* probs, hipStream_t s);
hipError_t batch_mstep(const BatchItem* items, int n, const BatchProblem* probs, int t, int K, double alpha_max,
                       hipStream_t s);
hipError_t batch_running(const BatchProblem* probs, int n, int32_t* out, hipStream_t s);

// ------------------------------------------------------------ learned form
void set_last_error(const std::string& msg);
cofem_status net_predict(cofem_net* n, const float* alpha, const float* alpha_prev, const double* mu_prev,
                         const float* s_prev, const float* taps, int ntaps, double beta, float* d0, double* mu0,
                         hipStream_t s);
cofem_status net_features(cofem_net* n, const float* alpha, const float* alpha_prev, const double* mu_prev,
                          const float* s_prev, const float* taps, int ntaps, double beta, float* feats, float* aux,
                          hipStream_t s);
int net_height(const cofem_net* n);
int net_width(const cofem_net* n);

}  // namespace cofem
