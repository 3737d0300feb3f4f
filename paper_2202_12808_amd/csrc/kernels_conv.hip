// 2D circular-convolution dictionary kernels of the CoFEM E-step.
//
// Phi is a circular convolution with an odd ks x ks kernel (a structured
// dictionary with a fast apply, Sec. 1 and Sec. 3.2 of arXiv 2202.12808):
//   (Phi z)[u, v]   = sum_{a,b} h[a,b] z[(u - a + c) mod H, (v - b + c) mod W]
//   (Phi^T w)[u, v] = sum_{a,b} h[a,b] w[(u + a - c) mod H, (v + b - c) mod W]
// with c = (ks - 1)/2.  The operator application
//   q = beta Phi^T (Phi p) + alpha (.) p
// runs as a single pass per output tile and column: the tile of p with a 2c
// halo is staged in LDS, Phi p is formed on the tile with a c halo in a
// second LDS buffer, and Phi^T of that gives q on the tile, each thread
// computing 4x4 output blocks.  The pass also forms gam = p^T q,
// del = r^T M^-1 q and eta = q^T M^-1 q.  The first CG iteration of a solve
// is that pass alone; each later one is a fused launch that applies the
// previous update (x += a p, r -= a q, p <- M^-1 r + b p) while it stages p
// and then runs the pass, so the state is streamed once per iteration.
//
// State layout: probe columns are column-major images (column k at k * ldD,
// pixel j = u * W + v) of type TP (float, or double in the float64 mode); the
// mean column is always a float64 image.
#include "conv_tile.h"

namespace cofem {

// The CG update that a fused iteration applies while it stages p: the
// previous iteration's p, r and q (read: a neighbouring tile's halo reads
// them too, so the new r and p go to the other buffer of a pair), x updated in
// place, the new r and p written for the tile's own pixels, and the step
// scalars of the column.
template <typename T>
struct FusedUpd {
  const T* P0;
  const T* R0;
  const T* Q0;
  T* X;
  T* P1;
  T* R1;
  T a, b;
};

// One output tile of one column of the fused operator pass, in precision T:
// q = beta Phi^T (Phi p) + alpha (.) p on the tile, written to Q, and the
// thread's parts of gam = p^T q, del = r^T M^-1 q, eta = q^T M^-1 q.
// `near` (uniform): every staged coordinate is within one period of the
// image, so wrapping is a compare and an add.
// FUSED: p is not read but formed while staging from the previous
// iteration's state (`fu`): r' = r - a q, z = M^-1 r', p' = z + b p (the
// textbook CG update's arithmetic), with x += a p, r' and p' written and
// dots[3..4] = r'^T z, r'^T r' summed for the tile's own pixels; R and P are
// then unused and the epilogue's r is r' recomputed from fu.R0 and fu.Q0.
template <int KS, int TILE, typename T, typename TapsT, bool FUSED = false>
__device__ __forceinline__ void conv_tile(TapsT h, int H, int W, int tu0, int tv0, bool near,
                                          const T* __restrict__ P, const T* __restrict__ R,
                                          const float* __restrict__ alpha, T beta,
                                          const float* __restrict__ minv, T* __restrict__ Q, T* sP, T* sT,
                                          double* dots, const FusedUpd<T>* fu = nullptr) {
  using G = ConvGeom<KS, TILE>;
  constexpr int c = G::c;
  const int tid = threadIdx.x;
  // stage 0: p on the tile plus a 2c halo (circular wrap).  Every load of
  // the thread is issued before the first LDS store, so the staging costs
  // about one memory latency, not one per element.
  if constexpr (FUSED) {
    constexpr int N0 = G::SPH * G::SPW, PER = (N0 + kThreads - 1) / kThreads, GRP = 7;
    const T a = fu->a, b = fu->b;
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int k0 = 0; k0 < PER; k0 += GRP) {
      T p0[GRP], r0[GRP], q0[GRP], x0[GRP];
      float mv[GRP];
      int64_t ix[GRP];
      bool ok[GRP], own[GRP];
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
        const int e = tid + (k0 + k) * kThreads;
        ok[k] = k0 + k < PER && e < N0;
        own[k] = false;
        if (ok[k]) {
          const int i = e / G::SPW, j = e - (e / G::SPW) * G::SPW;
          int u = tu0 - 2 * c + i, v = tv0 - 2 * c + j;
          // the tile's own pixels: unwrapped, inside the tile and the image
          own[k] = i >= 2 * c && i < 2 * c + TILE && j >= 2 * c && j < 2 * c + TILE && u < H && v < W;
          if (near) {
            u = u < 0 ? u + H : (u >= H ? u - H : u);
            v = v < 0 ? v + W : (v >= W ? v - W : v);
          } else {
            u = wrap(u, H);
            v = wrap(v, W);
          }
          ix[k] = (int64_t)u * W + v;
          p0[k] = fu->P0[ix[k]];
          r0[k] = fu->R0[ix[k]];
          q0[k] = fu->Q0[ix[k]];
          mv[k] = minv ? minv[ix[k]] : 1.0f;
          if (own[k]) x0[k] = fu->X[ix[k]];
        }
      }
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
        if (!ok[k]) continue;
        const T r1 = fma(-a, q0[k], r0[k]);
        const T z = minv ? (T)mv[k] * r1 : r1;
        const T p1 = fma(b, p0[k], z);
        sP[tid + (k0 + k) * kThreads] = p1;
        if (own[k]) {
          fu->X[ix[k]] = fma(a, p0[k], x0[k]);
          fu->R1[ix[k]] = r1;
          fu->P1[ix[k]] = p1;
          rz += (double)r1 * (double)z;
          rr += (double)r1 * (double)r1;
        }
      }
    }
    dots[3] = rz;
    dots[4] = rr;
  } else {
    constexpr int N0 = G::SPH * G::SPW, PER = (N0 + kThreads - 1) / kThreads;
    T pv[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * kThreads;
      if (e < N0) {
        const int i = e / G::SPW, j = e - (e / G::SPW) * G::SPW;
        int u = tu0 - 2 * c + i, v = tv0 - 2 * c + j;
        if (near) {
          u = u < 0 ? u + H : (u >= H ? u - H : u);
          v = v < 0 ? v + W : (v >= W ? v - W : v);
        } else {
          u = wrap(u, H);
          v = wrap(v, W);
        }
        pv[k] = P[(int64_t)u * W + v];
      }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * kThreads;
      if (e < N0) sP[e] = pv[k];
    }
  }
  __syncthreads();
  // stage 1: t = Phi p on the tile plus a c halo
  conv_stage1<KS, TILE, T>(h, sP, sT, tid, kThreads);
  __syncthreads();
  // stage 2: q = beta Phi^T t + alpha p on the tile
  double g = 0.0, dl = 0.0, et = 0.0;
  const int bi2 = tid / (TILE / 4), bj2 = tid - (tid / (TILE / 4)) * (TILE / 4);
  T acc[4][4];
  if (tid < G::NB2) conv_stage2<KS, TILE, T>(h, sT, tid, acc);
  __syncthreads();  // every thread is done reading t
  if (tid < G::NB2) {
    T* dst = sT + (4 * bi2) * TILE + 4 * bj2;  // Phi^T t of the tile, TILE x TILE
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) dst[r * TILE + cc] = acc[r][cc];
  }
  __syncthreads();
  // epilogue, one output per thread per step (coalesced rows):
  // q = beta Phi^T t + alpha p, and the dots.  The steps' loads are issued
  // in groups of 8 before their uses.
  constexpr int PER2 = TILE * TILE / kThreads, GRP = PER2 < 8 ? PER2 : 8;
#pragma unroll
  for (int k0 = 0; k0 < PER2; k0 += GRP) {
    float al[GRP], mv[GRP];
    T rv[GRP];
    int64_t ix[GRP];
    bool ok[GRP];
#pragma unroll
    for (int k = 0; k < GRP; ++k) {
      const int e = tid + (k0 + k) * kThreads;
      const int i = e / TILE, j = e - (e / TILE) * TILE;
      const int u = tu0 + i, v = tv0 + j;
      ok[k] = u < H && v < W;
      ix[k] = (int64_t)u * W + v;
      al[k] = ok[k] ? alpha[ix[k]] : 0.0f;
      if constexpr (FUSED)  // r' = r - a q, the value the staging wrote
        rv[k] = ok[k] ? fma(-fu->a, fu->Q0[ix[k]], fu->R0[ix[k]]) : T(0);
      else
        rv[k] = ok[k] ? R[ix[k]] : T(0);
      mv[k] = (ok[k] && minv) ? minv[ix[k]] : 1.0f;
    }
#pragma unroll
    for (int k = 0; k < GRP; ++k) {
      if (!ok[k]) continue;
      const int e = tid + (k0 + k) * kThreads;
      const int i = e / TILE, j = e - (e / TILE) * TILE;
      const T p = sP[(i + 2 * c) * G::SPW + j + 2 * c];
      const T q = fma(beta, sT[e], (T)al[k] * p);  // one rounding order in every kernel
      Q[ix[k]] = q;
      const double qd = (double)q;
      // with a diagonal preconditioner the step's dots are weighted by it:
      // delta = r^T M^-1 q, eta = q^T M^-1 q (mv = 1 without one)
      const double mq = (double)mv[k] * qd;
      g += (double)p * qd;
      dl += (double)rv[k] * mq;
      et += qd * mq;
    }
  }
  dots[0] = g;
  dots[1] = dl;
  dots[2] = et;
}

// Grid: x = 64 x 64 tile (in an order that gives each XCD a contiguous band
// of tiles, so halo rows shared by neighbouring tiles stay in one L2),
// z = column part.  z < 4: quadrant z of the float64 mean column; then S
// parts per probe column (S = 1 for float columns, 4 quadrants in the float64
// mode).  Column k's partial dots come from ntiles * S_k workgroups.
template <int KS, typename TP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_pass(
    const float* __restrict__ taps, int H, int W, int64_t ldD, int K, int tilesX, const TP* __restrict__ P,
    const double* __restrict__ pm, const TP* __restrict__ R, const double* __restrict__ rm,
    const float* __restrict__ alpha, double beta, const float* __restrict__ minv, TP* __restrict__ Q,
    double* __restrict__ qm, ConvReduce red, int64_t nblk_alloc, int nt, CgScalars* __restrict__ st,
    int apply_only) {
  if (!apply_only && st->stop) return;
  const CgCtl ctl = load_cg_ctl(st);
  using G64 = ConvGeom<KS, kConvTile>;
  using G32 = ConvGeom<KS, kConvTile / 2>;
  constexpr int kS = sizeof(TP) == 8 ? 4 : 1;  // parts per probe column
  // float64 columns (the mean, and every column in the float64 mode) take
  // 32 x 32 quadrants; float columns 64 x 64 tiles
  constexpr size_t kBytes = kS == 4 ? G32::LDS * sizeof(double)
                                    : (G64::LDS * sizeof(float) > G32::LDS * sizeof(double) ? G64::LDS * sizeof(float)
                                                                                             : G32::LDS * sizeof(double));
  __shared__ __align__(16) unsigned char sbuf[kBytes];
  __shared__ double sTapsD[KS * KS];
  __shared__ float sTapsF[KS * KS];
  if (threadIdx.x < KS * KS) {
    sTapsD[threadIdx.x] = (double)taps[threadIdx.x];
    sTapsF[threadIdx.x] = taps[threadIdx.x];
  }
  __syncthreads();
  const int64_t ntiles = gridDim.x;
  int64_t tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (tile & 7) * (ntiles >> 3) + (tile >> 3);
  const int ty = (int)(tile / tilesX), tx = (int)(tile - (tile / tilesX) * tilesX);
  // z < 4 nt: quadrant z % 4 of mean column z / 4 (column K + z / 4); then
  // the probe columns' parts
  const int z = blockIdx.z;
  int col, part, nparts;
  if (z < 4 * nt) {
    col = K + (z >> 2);
    part = z & 3;
    nparts = 4;
  } else {
    col = (z - 4 * nt) / kS;
    part = (z - 4 * nt) - col * kS;
    nparts = kS;
  }
  int tu0 = ty * kConvTile, tv0 = tx * kConvTile;
  double dots[3];
  dots[0] = dots[1] = dots[2] = 0.0;
  if (nparts == 4) {  // a float64 quadrant
    tu0 += (part >> 1) * (kConvTile / 2);
    tv0 += (part & 1) * (kConvTile / 2);
  }
  if (tu0 >= H || tv0 >= W) {
    // a quadrant past the image edge: no outputs, zero dots (it still
    // arrives at the reduction)
  } else if (nparts == 4) {
    const bool near = H >= G32::TR && W >= G32::SPW - 2 * G32::c;
    double* sb = reinterpret_cast<double*>(sbuf);
    Taps<double> hd(sTapsD);
    if (col >= K) {
      const int64_t mo = (int64_t)(col - K) * ldD;
      conv_tile<KS, kConvTile / 2, double>(hd, H, W, tu0, tv0, near, pm + mo, rm + mo, alpha, beta, minv, qm + mo,
                                           sb, sb + G32::SPH * G32::SPW, dots);
    } else {
      const int64_t off = (int64_t)col * ldD;
      conv_tile<KS, kConvTile / 2, double>(hd, H, W, tu0, tv0, near, reinterpret_cast<const double*>(P) + off,
                                           reinterpret_cast<const double*>(R) + off, alpha, beta, minv,
                                           reinterpret_cast<double*>(Q) + off, sb, sb + G32::SPH * G32::SPW,
                                           dots);
    }
  } else if constexpr (kS == 1) {  // a float column's 64 x 64 tile
    const bool near = H >= G64::TR && W >= G64::SPW - 2 * G64::c;
    float* sb = reinterpret_cast<float*>(sbuf);
    Taps<float> hf(sTapsF);
    const int64_t off = (int64_t)col * ldD;
    conv_tile<KS, kConvTile, float>(hf, H, W, tu0, tv0, near, reinterpret_cast<const float*>(P) + off,
                                    reinterpret_cast<const float*>(R) + off, alpha, (float)beta, minv,
                                    reinterpret_cast<float*>(Q) + off, sb, sb + G64::SPH * G64::SPW, dots);
  }
  if (apply_only) return;
  __shared__ double shm[8];
  __shared__ double mine[3], tot[3 * kMaxCols];
  const double tg = block_sum(dots[0], shm);
  const double td = block_sum(dots[1], shm);
  const double te = block_sum(dots[2], shm);
  if (threadIdx.x == 0) {
    mine[0] = tg;
    mine[1] = td;
    mine[2] = te;
  }
  __syncthreads();
  if (!column_tree_reduce(red.parts, red.cnts, red.colsum, red.cnt_cols, tile * nparts + part, ntiles * nparts,
                          nblk_alloc, col, K + nt, 3, mine, tot))
    return;
  finish_step(st, tot, ctl);
}

// ------------------------------------------------ fused CG iteration
// One launch per CG iteration after the first: the update of the previous
// iteration (x += a p, r -= a q, z = M^-1 r, p = z + b p) applied while p is
// staged, then the operator pass on the new p, with the update's r^T z and
// r^T r and the pass's gam, del, eta reduced together.  Its finish applies
// the stop test on ||r||_F and, if the solve goes on, sets the next step's a
// and b -- the same arithmetic and decisions as a separate update followed by
// a pass, with the update's stream of the state overlapped with the
// stencil's arithmetic (a solve's last launch computes one operator product
// that is not used).  p, r, q alternate between two buffers (a tile's halo
// reads its neighbours' old values while they write their new ones); x is
// updated in place.  The grid is the operator pass's.
template <int KS, typename TP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_fused(
    const float* __restrict__ taps, int H, int W, int64_t ldD, int K, int tilesX, const TP* __restrict__ P0,
    const TP* __restrict__ R0, const TP* __restrict__ Q0, TP* __restrict__ X, TP* __restrict__ P1,
    TP* __restrict__ R1, TP* __restrict__ Q1, const double* __restrict__ pm0, const double* __restrict__ rm0,
    const double* __restrict__ qm0, double* __restrict__ xm, double* __restrict__ pm1, double* __restrict__ rm1,
    double* __restrict__ qm1, const float* __restrict__ alpha, double beta, const float* __restrict__ minv,
    ConvReduce red, int64_t nblk_alloc, int nt, CgScalars* __restrict__ st) {
  if (st->stop) return;
  const CgCtl ctl = load_cg_ctl(st);
  using G64 = ConvGeom<KS, kConvTile>;
  using G32 = ConvGeom<KS, kConvTile / 2>;
  constexpr int kS = sizeof(TP) == 8 ? 4 : 1;  // parts per probe column
  constexpr size_t kBytes = kS == 4 ? G32::LDS * sizeof(double)
                                    : (G64::LDS * sizeof(float) > G32::LDS * sizeof(double) ? G64::LDS * sizeof(float)
                                                                                             : G32::LDS * sizeof(double));
  __shared__ __align__(16) unsigned char sbuf[kBytes];
  __shared__ double sTapsD[KS * KS];
  __shared__ float sTapsF[KS * KS];
  if (threadIdx.x < KS * KS) {
    sTapsD[threadIdx.x] = (double)taps[threadIdx.x];
    sTapsF[threadIdx.x] = taps[threadIdx.x];
  }
  __syncthreads();
  const int64_t ntiles = gridDim.x;
  int64_t tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (tile & 7) * (ntiles >> 3) + (tile >> 3);
  const int ty = (int)(tile / tilesX), tx = (int)(tile - (tile / tilesX) * tilesX);
  const int z = blockIdx.z;
  int col, part, nparts;
  if (z < 4 * nt) {
    col = K + (z >> 2);
    part = z & 3;
    nparts = 4;
  } else {
    col = (z - 4 * nt) / kS;
    part = (z - 4 * nt) - col * kS;
    nparts = kS;
  }
  int tu0 = ty * kConvTile, tv0 = tx * kConvTile;
  double dots[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (nparts == 4) {
    tu0 += (part >> 1) * (kConvTile / 2);
    tv0 += (part & 1) * (kConvTile / 2);
  }
  if (tu0 >= H || tv0 >= W) {
    // a quadrant past the image edge: no pixels, zero sums
  } else if (nparts == 4) {
    const bool near = H >= G32::TR && W >= G32::SPW - 2 * G32::c;
    double* sb = reinterpret_cast<double*>(sbuf);
    Taps<double> hd(sTapsD);
    const double a = st->a[col], b = st->b[col];
    if (col >= K) {
      const int64_t mo = (int64_t)(col - K) * ldD;
      const FusedUpd<double> fu{pm0 + mo, rm0 + mo, qm0 + mo, xm + mo, pm1 + mo, rm1 + mo, a, b};
      conv_tile<KS, kConvTile / 2, double, Taps<double>, true>(hd, H, W, tu0, tv0, near, nullptr, nullptr, alpha,
                                                               beta, minv, qm1 + mo, sb, sb + G32::SPH * G32::SPW,
                                                               dots, &fu);
    } else {
      const int64_t off = (int64_t)col * ldD;
      const double* dP0 = reinterpret_cast<const double*>(P0) + off;
      const double* dR0 = reinterpret_cast<const double*>(R0) + off;
      const double* dQ0 = reinterpret_cast<const double*>(Q0) + off;
      const FusedUpd<double> fu{dP0, dR0, dQ0, reinterpret_cast<double*>(X) + off,
                                reinterpret_cast<double*>(P1) + off, reinterpret_cast<double*>(R1) + off, a, b};
      conv_tile<KS, kConvTile / 2, double, Taps<double>, true>(hd, H, W, tu0, tv0, near, nullptr, nullptr, alpha,
                                                               beta, minv, reinterpret_cast<double*>(Q1) + off, sb,
                                                               sb + G32::SPH * G32::SPW, dots, &fu);
    }
  } else if constexpr (kS == 1) {  // a float column's 64 x 64 tile
    const bool near = H >= G64::TR && W >= G64::SPW - 2 * G64::c;
    float* sb = reinterpret_cast<float*>(sbuf);
    Taps<float> hf(sTapsF);
    const int64_t off = (int64_t)col * ldD;
    const FusedUpd<float> fu{reinterpret_cast<const float*>(P0) + off, reinterpret_cast<const float*>(R0) + off,
                             reinterpret_cast<const float*>(Q0) + off, reinterpret_cast<float*>(X) + off,
                             reinterpret_cast<float*>(P1) + off, reinterpret_cast<float*>(R1) + off,
                             (float)st->a[col], (float)st->b[col]};
    conv_tile<KS, kConvTile, float, Taps<float>, true>(hf, H, W, tu0, tv0, near, nullptr, nullptr, alpha,
                                                       (float)beta, minv, reinterpret_cast<float*>(Q1) + off, sb,
                                                       sb + G64::SPH * G64::SPW, dots, &fu);
  }
  __shared__ double shm[8];
  __shared__ double mine[5], tot[5 * kMaxCols];
  // r^T z, r^T r, gam, del, eta
  const double v0 = block_sum(dots[3], shm);
  const double v1 = block_sum(dots[4], shm);
  const double v2 = block_sum(dots[0], shm);
  const double v3 = block_sum(dots[1], shm);
  const double v4 = block_sum(dots[2], shm);
  if (threadIdx.x == 0) {
    mine[0] = v0;
    mine[1] = v1;
    mine[2] = v2;
    mine[3] = v3;
    mine[4] = v4;
  }
  __syncthreads();
  if (!column_tree_reduce(red.parts, red.cnts, red.colsum, red.cnt_cols, tile * nparts + part, ntiles * nparts,
                          nblk_alloc, col, K + nt, 5, mine, tot))
    return;
  finish_fused(st, tot, K + nt, ctl);
}

template <typename TP>
static hipError_t launch_conv_fused(const ConvDims& cd, const float* taps, const ConvState& s0, const ConvState& s1,
                                    void* X, double* xm, const float* alpha, double beta, const float* minv,
                                    const ConvReduce& red, CgScalars* st, hipStream_t s) {
  constexpr int kS = sizeof(TP) == 8 ? 4 : 1;
  const dim3 grid((unsigned)(cd.tilesX * cd.tilesY), 1, (unsigned)(4 * cd.nt + cd.K * kS));
  const int64_t nblk_alloc = conv_pass_blocks(cd);
#define COFEM_FUSED_CASE(KS)                                                                                    \
  case KS:                                                                                                      \
    hipLaunchKernelGGL((k_conv_fused<KS, TP>), grid, dim3(kThreads), 0, s, taps, cd.H, cd.W, cd.ldD, cd.K,        \
                       cd.tilesX, static_cast<const TP*>(s0.P), static_cast<const TP*>(s0.R),                     \
                       static_cast<const TP*>(s0.Q), static_cast<TP*>(X), static_cast<TP*>(s1.P),                  \
                       static_cast<TP*>(s1.R), static_cast<TP*>(s1.Q), s0.pm, s0.rm, s0.qm, xm, s1.pm, s1.rm,      \
                       s1.qm, alpha, beta, minv, red, nblk_alloc, cd.nt, st);                                     \
    break;
  switch (cd.ks) {
    COFEM_FUSED_CASE(1)
    COFEM_FUSED_CASE(3)
    COFEM_FUSED_CASE(5)
    COFEM_FUSED_CASE(7)
    COFEM_FUSED_CASE(9)
    default:
      return hipErrorInvalidValue;
  }
#undef COFEM_FUSED_CASE
  return hipGetLastError();
}

hipError_t conv_fused(const ConvDims& cd, const float* taps, const ConvState& s0, const ConvState& s1, void* X,
                      double* xm, const float* alpha, double beta, const float* minv, const ConvReduce& red,
                      CgScalars* st, hipStream_t s) {
  if (cd.ws_grid > 0) return conv_fused_ws(cd, cd.ws_grid, taps, s0, s1, X, xm, alpha, beta, minv, red, st, s);
  if (cd.fp64) return launch_conv_fused<double>(cd, taps, s0, s1, X, xm, alpha, beta, minv, red, st, s);
  return launch_conv_fused<float>(cd, taps, s0, s1, X, xm, alpha, beta, minv, red, st, s);
}

template <typename TP>
static hipError_t launch_conv_pass(const ConvDims& cd, const float* taps, const void* P,
                                   const double* pm, const void* R, const double* rm,
                                   const float* alpha, double beta, const float* minv, void* Q, double* qm,
                                   const ConvReduce& red, CgScalars* st, int apply_only, hipStream_t s) {
  constexpr int kS = sizeof(TP) == 8 ? 4 : 1;
  const dim3 grid((unsigned)(cd.tilesX * cd.tilesY), 1, (unsigned)(4 * cd.nt + cd.K * kS));
  const TP* Pt = static_cast<const TP*>(P);
  const TP* Rt = static_cast<const TP*>(R);
  TP* Qt = static_cast<TP*>(Q);
  const int64_t nblk_alloc = conv_pass_blocks(cd);
#define COFEM_CONV_CASE(KS)                                                                             \
  case KS:                                                                                              \
    hipLaunchKernelGGL((k_conv_pass<KS, TP>), grid, dim3(kThreads), 0, s, taps, cd.H, cd.W, cd.ldD, cd.K,  \
                       cd.tilesX, Pt, pm, Rt, rm, alpha, beta, minv, Qt, qm, red, nblk_alloc, cd.nt, st,      \
                       apply_only);                                                                     \
    break;
  switch (cd.ks) {
    COFEM_CONV_CASE(1)
    COFEM_CONV_CASE(3)
    COFEM_CONV_CASE(5)
    COFEM_CONV_CASE(7)
    COFEM_CONV_CASE(9)
    default:
      return hipErrorInvalidValue;
  }
#undef COFEM_CONV_CASE
  return hipGetLastError();
}

hipError_t conv_pass(const ConvDims& cd, const float* taps, const void* P, const double* pm,
                     const void* R, const double* rm, const float* alpha, double beta, void* Q,
                     double* qm, const ConvReduce& red, CgScalars* st, int apply_only, hipStream_t s,
                     const float* minv) {
  if (cd.ws_grid > 0) return conv_pass_ws(cd, cd.ws_grid, taps, P, pm, R, rm, alpha, beta, Q, qm, red, st, apply_only, s, minv);
  if (cd.fp64)
    return launch_conv_pass<double>(cd, taps, P, pm, R, rm, alpha, beta, minv, Q, qm, red, st, apply_only, s);
  return launch_conv_pass<float>(cd, taps, P, pm, R, rm, alpha, beta, minv, Q, qm, red, st, apply_only, s);
}

// Workgroups whose partial dots one column of the operator pass may reduce
// (the reduction workspace is sized for this many per column).
int64_t conv_pass_blocks(const ConvDims& cd) { return 4 * (int64_t)cd.tilesX * cd.tilesY; }

// ------------------------------------------------ b0 = beta Phi^T y (Eq. 5), float64
__global__ void k_conv_b0(const float* __restrict__ taps, int ks, int H, int W, int64_t ldD,
                          const float* __restrict__ y, double beta, double* __restrict__ b0) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ldD) return;
  const int64_t D = (int64_t)H * W;
  if (d >= D) {
    b0[d] = 0.0;
    return;
  }
  const int u = (int)(d / W), v = (int)(d % W), c = (ks - 1) / 2;
  double acc = 0.0;
  for (int a = 0; a < ks; ++a)
    for (int b = 0; b < ks; ++b)
      acc = fma((double)taps[a * ks + b], (double)y[(int64_t)wrap(u + a - c, H) * W + wrap(v + b - c, W)], acc);
  b0[d] = beta * acc;
}

hipError_t conv_b0(const ConvDims& cd, const float* taps, const float* y, double beta, double* b0,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_conv_b0, dim3((unsigned)((cd.ldD + 255) / 256)), dim3(256), 0, s, taps, cd.ks,
                     cd.H, cd.W, cd.ldD, y, beta, b0);
  return hipGetLastError();
}

int conv_update_blocks(const ConvDims& cd) {
  const int64_t want = (cd.D + 4 * 256 - 1) / (4 * 256);
  return (int)(want < 1 ? 1 : (want > 256 ? 256 : want));
}

// ------------------------------------------------ initial residual R = P = B (Eq. 7)
template <typename TP>
__global__ __launch_bounds__(256) void k_conv_init(int64_t D, int64_t ldD, int K, int perm, int nt, uint64_t seed,
                                                   int t, const double* __restrict__ b0,
                                                   TP* __restrict__ X, TP* __restrict__ R,
                                                   TP* __restrict__ P, double* __restrict__ xm,
                                                   double* __restrict__ rm, double* __restrict__ pm,
                                                   ConvReduce red, CgScalars* st) {
  const int col = blockIdx.y;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  if (col >= K) {  // mean column col - K
    const int64_t mo = (int64_t)(col - K) * ldD;
    for (int64_t d = gtid; d < D; d += gstride) {
      const double b = b0[mo + d];
      rm[mo + d] = b;
      pm[mo + d] = b;
      xm[mo + d] = 0.0;
      acc += b * b;
    }
  } else {
    const int64_t off = (int64_t)col * ldD;
    for (int64_t d = gtid; d < D; d += gstride) {
      const TP v = (TP)probe_sign(seed, (uint32_t)t, (uint32_t)col, (uint64_t)perm_nat(perm, d));
      R[off + d] = v;
      P[off + d] = v;
      X[off + d] = TP(0);
      acc += 1.0;
    }
  }
  __shared__ double shm[8];
  __shared__ double mine[1], tot[kMaxCols];
  const double tot_b = block_sum(acc, shm);
  if (threadIdx.x == 0) mine[0] = tot_b;
  __syncthreads();
  if (!column_tree_reduce(red.parts, red.cnts, red.colsum, red.cnt_cols, blockIdx.x, gridDim.x, col,
                          K + nt, 1, mine, tot))
    return;
  finish_init(st, tot);
}

hipError_t conv_init(const ConvDims& cd, uint64_t seed, int t, const double* b0, void* X, void* R,
                     void* P, double* xm, double* rm, double* pm, const ConvReduce& red,
                     CgScalars* st, hipStream_t s) {
  const dim3 grid(conv_update_blocks(cd), cd.K + cd.nt);
  if (cd.fp64)
    hipLaunchKernelGGL(k_conv_init<double>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, b0,
                       static_cast<double*>(X), static_cast<double*>(R), static_cast<double*>(P), xm,
                       rm, pm, red, st);
  else
    hipLaunchKernelGGL(k_conv_init<float>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, b0,
                       static_cast<float*>(X), static_cast<float*>(R), static_cast<float*>(P), xm, rm,
                       pm, red, st);
  return hipGetLastError();
}

// ------------------------------------------------ preconditioned CG from a starting block
// (warm-started and learned forms).  M^-1 = diag(minv) for every column (null:
// identity).  With a start X0 (already in X / xm) and Q = A X0 from an
// operator pass: R = B - Q; without one: R = B, X = 0.  Then Z = M^-1 R,
// P = Z; per column rho = r^T z, ||r||^2 (the stop test's) and ||b||^2.
template <typename TP>
__global__ __launch_bounds__(256) void k_conv_init_pcg(int64_t D, int64_t ldD, int K, int perm, int nt, uint64_t seed,
                                                       int t,
                                                       const double* __restrict__ b0, const float* __restrict__ minv,
                                                       const TP* __restrict__ Qx, const double* __restrict__ qxm,
                                                       TP* __restrict__ X, TP* __restrict__ R, TP* __restrict__ P,
                                                       double* __restrict__ xm, double* __restrict__ rm,
                                                       double* __restrict__ pm, ConvReduce red, CgScalars* st) {
  const int col = blockIdx.y;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (col >= K) {  // mean column col - K
    const int64_t mo = (int64_t)(col - K) * ldD;
    for (int64_t d = gtid; d < D; d += gstride) {
      const double b = b0[mo + d];
      const double r = qxm ? b - qxm[mo + d] : b;
      const double z = minv ? (double)minv[d] * r : r;
      rm[mo + d] = r;
      pm[mo + d] = z;
      if (!qxm) xm[mo + d] = 0.0;
      rz += r * z;
      rr += r * r;
      bb += b * b;
    }
  } else {
    // four pixels per pass, their loads issued together (the same per-pixel
    // arithmetic and summation order as one at a time)
    constexpr int G = 4;
    const int64_t off = (int64_t)col * ldD;
    for (int64_t d0 = gtid; d0 < D; d0 += G * gstride) {
      TP qv[G];
      float mv[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int64_t d = d0 + g * gstride;
        qv[g] = (Qx && d < D) ? Qx[off + d] : TP(0);
        mv[g] = (minv && d < D) ? minv[d] : 1.0f;
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int64_t d = d0 + g * gstride;
        if (d >= D) continue;
        const TP b = (TP)probe_sign(seed, (uint32_t)t, (uint32_t)col, (uint64_t)perm_nat(perm, d));
        const TP r = Qx ? b - qv[g] : b;
        const TP z = minv ? (TP)mv[g] * r : r;
        R[off + d] = r;
        P[off + d] = z;
        if (!Qx) X[off + d] = TP(0);
        rz += (double)r * (double)z;
        rr += (double)r * (double)r;
        bb += 1.0;
      }
    }
  }
  __shared__ double shm[8];
  __shared__ double mine[3], tot[3 * kMaxCols];
  const double v0 = block_sum(rz, shm);
  const double v1 = block_sum(rr, shm);
  const double v2 = block_sum(bb, shm);
  if (threadIdx.x == 0) {
    mine[0] = v0;
    mine[1] = v1;
    mine[2] = v2;
  }
  __syncthreads();
  if (!column_tree_reduce(red.parts, red.cnts, red.colsum, red.cnt_cols, blockIdx.x, gridDim.x, col, K + nt, 3, mine,
                          tot))
    return;
  finish_init_pcg(st, tot, K + nt);
}

hipError_t conv_init_pcg(const ConvDims& cd, uint64_t seed, int t, const double* b0, const float* minv,
                         const void* Qx, const double* qxm, void* X, void* R, void* P, double* xm, double* rm,
                         double* pm, const ConvReduce& red, CgScalars* st, hipStream_t s) {
  const dim3 grid(conv_update_blocks(cd), cd.K + cd.nt);
  if (cd.fp64)
    hipLaunchKernelGGL(k_conv_init_pcg<double>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, b0,
                       minv,
                       static_cast<const double*>(Qx), qxm, static_cast<double*>(X), static_cast<double*>(R),
                       static_cast<double*>(P), xm, rm, pm, red, st);
  else
    hipLaunchKernelGGL(k_conv_init_pcg<float>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, b0,
                       minv,
                       static_cast<const float*>(Qx), qxm, static_cast<float*>(X), static_cast<float*>(R),
                       static_cast<float*>(P), xm, rm, pm, red, st);
  return hipGetLastError();
}

// Starting block X0 = [max(d0, 0) (.) p_1 .. max(d0, 0) (.) p_K | mu0] (d0 null:
// zero probe columns; mu0 null: keep xm as it is, the previous solve's mean
// column).
// Grid: x over the pixels, y over the columns (no 64-bit division per element).
template <typename TP>
__global__ void k_conv_start(int64_t D, int64_t ldD, int K, int perm, int nt, uint64_t seed, int t,
                             const float* __restrict__ d0, const double* __restrict__ mu0, TP* __restrict__ X,
                             double* __restrict__ xm) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (k >= K) {  // mean column k - K
    if (d < D && mu0) xm[(k - K) * ldD + d] = mu0[(k - K) * ldD + d];
    return;
  }
  float sg;
  if (perm == 0) {
    // natural order: a wave's 64 pixels (from a multiple of 64, d & 63 =
    // lane) share one SplitMix64 word of probe k, formed once per wave
    const uint64_t j6 = (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)d >> 6));
    const uint64_t idx = ((uint64_t)t << 48) | ((uint64_t)k << 32) | j6;
    const uint64_t w = splitmix64_mix(seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
    sg = ((w >> (d & 63)) & 1ull) ? -1.0f : 1.0f;
  } else {
    sg = probe_sign(seed, (uint32_t)t, (uint32_t)k, (uint64_t)perm_nat(perm, d));
  }
  if (d >= D) return;
  const float dv = d0 ? fmaxf(d0[d], 0.0f) : 0.0f;
  X[k * ldD + d] = (TP)(dv * sg);
}

// The same start, four pixels per thread with 16-byte accesses (natural
// order, D and ldD multiples of 4): a quarter of the blocks, and one
// SplitMix64 word per thread (its four signs are bits d & 63 .. + 3).
template <typename TP>
__global__ void k_conv_start4(int64_t D, int64_t ldD, int K, uint64_t seed, int t, const float* __restrict__ d0,
                              const double* __restrict__ mu0, TP* __restrict__ X, double* __restrict__ xm) {
  const int64_t d = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  const int64_t k = blockIdx.y;
  if (d >= D) return;
  if (k >= K) {  // mean column k - K
    if (mu0) {
      const double2* src = reinterpret_cast<const double2*>(mu0 + (k - K) * ldD + d);
      double2* dst = reinterpret_cast<double2*>(xm + (k - K) * ldD + d);
      const double2 a = src[0], b = src[1];
      dst[0] = a;
      dst[1] = b;
    }
    return;
  }
  const uint64_t idx = ((uint64_t)t << 48) | ((uint64_t)k << 32) | ((uint64_t)d >> 6);
  const uint32_t bits = (uint32_t)(splitmix64_mix(seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull) >> (d & 63));
  float4 dv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (d0) dv = *reinterpret_cast<const float4*>(d0 + d);
  const float x0 = fmaxf(dv.x, 0.0f) * ((bits & 1u) ? -1.0f : 1.0f);
  const float x1 = fmaxf(dv.y, 0.0f) * ((bits & 2u) ? -1.0f : 1.0f);
  const float x2 = fmaxf(dv.z, 0.0f) * ((bits & 4u) ? -1.0f : 1.0f);
  const float x3 = fmaxf(dv.w, 0.0f) * ((bits & 8u) ? -1.0f : 1.0f);
  TP* out = X + k * ldD + d;
  if constexpr (sizeof(TP) == 4) {
    *reinterpret_cast<float4*>(out) = make_float4(x0, x1, x2, x3);
  } else {
    reinterpret_cast<double2*>(out)[0] = make_double2(x0, x1);
    reinterpret_cast<double2*>(out)[1] = make_double2(x2, x3);
  }
}

hipError_t conv_start(const ConvDims& cd, uint64_t seed, int t, const float* d0, const double* mu0, void* X,
                      double* xm, hipStream_t s) {
  if (cd.perm == 0 && cd.D % 4 == 0 && cd.ldD % 4 == 0) {
    const dim3 grid4((unsigned)((cd.D / 4 + 255) / 256), (unsigned)(cd.K + cd.nt));
    if (cd.fp64)
      hipLaunchKernelGGL(k_conv_start4<double>, grid4, dim3(256), 0, s, cd.D, cd.ldD, cd.K, seed, t, d0, mu0,
                         static_cast<double*>(X), xm);
    else
      hipLaunchKernelGGL(k_conv_start4<float>, grid4, dim3(256), 0, s, cd.D, cd.ldD, cd.K, seed, t, d0, mu0,
                         static_cast<float*>(X), xm);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((cd.D + 255) / 256), (unsigned)(cd.K + cd.nt));
  if (cd.fp64)
    hipLaunchKernelGGL(k_conv_start<double>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, d0, mu0,
                       static_cast<double*>(X), xm);
  else
    hipLaunchKernelGGL(k_conv_start<float>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, d0, mu0,
                       static_cast<float*>(X), xm);
  return hipGetLastError();
}

// Jacobi: minv_j = 1 / (beta ||h||^2 + alpha_j) (every column of Phi has norm ||h||).
__global__ void k_conv_jacobi(int64_t D, const float* __restrict__ taps, int ntaps, double beta,
                              const float* __restrict__ alpha, float* __restrict__ minv) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  const double hh = taps_sq_sum(taps, ntaps);
  minv[d] = (float)(1.0 / (beta * hh + (double)alpha[d]));
}

hipError_t conv_jacobi(const ConvDims& cd, const float* taps, double beta, const float* alpha, float* minv,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_conv_jacobi, dim3((unsigned)((cd.D + 255) / 256)), dim3(256), 0, s, cd.D, taps,
                     cd.ks * cd.ks, beta, alpha, minv);
  return hipGetLastError();
}

// ------------------------------------------------ true residual (final check of a solve)
// ||b_c - q_c||^2 per column with q = A x from an operator pass over X and B
// regenerated: probes of EM iteration t (Eq. 7) and b0 for the mean column.
template <typename TP>
__global__ __launch_bounds__(256) void k_conv_true_resid(int64_t D, int64_t ldD, int K, int perm, int nt, uint64_t seed,
                                                         int t, const double* __restrict__ b0,
                                                         const TP* __restrict__ Q,
                                                         const double* __restrict__ qm, ConvReduce red,
                                                         CgScalars* st) {
  const int col = blockIdx.y;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  if (col >= K) {  // mean column col - K
    const int64_t mo = (int64_t)(col - K) * ldD;
    for (int64_t d = gtid; d < D; d += gstride) {
      const double e = b0[mo + d] - qm[mo + d];
      acc += e * e;
    }
  } else {
    const TP* q = Q + (int64_t)col * ldD;
    for (int64_t d = gtid; d < D; d += gstride) {
      const double e =
          (double)probe_sign(seed, (uint32_t)t, (uint32_t)col, (uint64_t)perm_nat(perm, d)) - (double)q[d];
      acc += e * e;
    }
  }
  __shared__ double shm[8];
  __shared__ double mine[1], tot[kMaxCols];
  const double tot_b = block_sum(acc, shm);
  if (threadIdx.x == 0) mine[0] = tot_b;
  __syncthreads();
  if (!column_tree_reduce(red.parts, red.cnts, red.colsum, red.cnt_cols, blockIdx.x, gridDim.x, col,
                          K + nt, 1, mine, tot))
    return;
  finish_true_resid(st, tot);
}

hipError_t conv_true_resid(const ConvDims& cd, uint64_t seed, int t, const double* b0, const void* Q,
                           const double* qm, const ConvReduce& red, CgScalars* st, hipStream_t s) {
  const dim3 grid(conv_update_blocks(cd), cd.K + cd.nt);
  if (cd.fp64)
    hipLaunchKernelGGL(k_conv_true_resid<double>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, b0,
                       static_cast<const double*>(Q), qm, red, st);
  else
    hipLaunchKernelGGL(k_conv_true_resid<float>, grid, dim3(256), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t, b0,
                       static_cast<const float*>(Q), qm, red, st);
  return hipGetLastError();
}

// ------------------------------------------------ diagonal estimate + M-step (Eq. 6, Eq. 8)
// 1024 threads per block (conv_update_blocks blocks), each taking its pixels
// kMsGroup at a time: the group's probe-column loads are issued together, so
// a thread has 4 K loads in flight instead of K (the launch is one block per
// compute unit, and with one pixel at a time it waited on every load).
constexpr int kMsThreads = 1024, kMsGroup = 4;
template <typename TP>
__global__ __launch_bounds__(kMsThreads) void k_conv_mstep(int64_t D, int64_t ldD, int K, int perm, int nt,
                                                           uint64_t seed, int t, const TP* __restrict__ X,
                                                           const double* __restrict__ xm,
                                                           float* __restrict__ alpha, double alpha_max,
                                                           float* __restrict__ mu,
                                                           float* __restrict__ sdiag, double* parts, uint32_t* cnts,
                                                           CgScalars* st, float* __restrict__ alpha_prev) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  const double floor_v = 1.0 / alpha_max;
  double clamped = 0.0, dg2 = 0.0, g2 = 0.0;
  // the loop test is uniform across a wave (its first pixel), so every lane
  // takes part in the shared hashing below; each pixel is guarded on its own
  for (int64_t d0 = gtid; (d0 & ~(int64_t)63) < D; d0 += kMsGroup * gstride) {
    double acc[kMsGroup];
#pragma unroll
    for (int g = 0; g < kMsGroup; ++g) acc[g] = 0.0;
    // In the natural element order a wave's 64 pixels d (a multiple of 64
    // onwards, d & 63 = lane) share probe k's 64-bit SplitMix64 word (the sign
    // is its bit d & 63): lane k forms the word of probe k once, and the wave
    // reads it from that lane, instead of every lane hashing all K words.
    uint64_t wk[kMsGroup];
    const int lane = threadIdx.x & 63;
    if (perm == 0) {
#pragma unroll
      for (int g = 0; g < kMsGroup; ++g) {
        const uint64_t idx = ((uint64_t)t << 48) | ((uint64_t)lane << 32) | ((uint64_t)(d0 + g * gstride) >> 6);
        wk[g] = splitmix64_mix(seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
      }
    }
    // the K probe columns in order for every pixel of the group (the same
    // summation order as one pixel at a time); loads unconditional (a pixel
    // past D reads pixel D - 1; its sum is never used) so that several
    // columns' loads are in flight
    int64_t dc[kMsGroup];
#pragma unroll
    for (int g = 0; g < kMsGroup; ++g) {
      const int64_t d = d0 + g * gstride;
      dc[g] = d < D ? d : D - 1;
    }
    if (perm == 0) {
      auto add = [&](int k, const TP* x) {
#pragma unroll
        for (int g = 0; g < kMsGroup; ++g) {
          const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)wk[g], k);
          const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(wk[g] >> 32), k);
          const uint64_t w = ((uint64_t)hi << 32) | lo;
          const float sg = ((w >> lane) & 1ull) ? -1.0f : 1.0f;
          acc[g] += (double)sg * (double)x[g];
        }
      };
      int k = 0;
      for (; k + 4 <= K; k += 4) {  // four columns' loads first, then their sums in order
        TP x[4][kMsGroup];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int g = 0; g < kMsGroup; ++g) x[u][g] = X[(int64_t)(k + u) * ldD + dc[g]];
#pragma unroll
        for (int u = 0; u < 4; ++u) add(k + u, x[u]);
      }
      for (; k < K; ++k) {
        TP x[kMsGroup];
#pragma unroll
        for (int g = 0; g < kMsGroup; ++g) x[g] = X[(int64_t)k * ldD + dc[g]];
        add(k, x);
      }
    } else {
      for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int g = 0; g < kMsGroup; ++g) {
          const float sg = probe_sign(seed, (uint32_t)t, (uint32_t)k, (uint64_t)perm_nat(perm, dc[g]));
          acc[g] += (double)sg * (double)X[(int64_t)k * ldD + dc[g]];
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kMsGroup; ++g) {
      const int64_t d = d0 + g * gstride;
      if (d >= D) continue;
      const double s = acc[g] / (double)K;
      const double m = xm[d];
      // tasks sharing alpha: the mean of their squared means
      double m2 = m * m;
      if (nt > 1) {
        for (int j = 1; j < nt; ++j) {
          const double mj = xm[(int64_t)j * ldD + d];
          m2 += mj * mj;
        }
        m2 /= (double)nt;
      }
      const double den = m2 + s;
      if (!(den >= floor_v)) clamped += 1.0;
      const float a_new = (float)(1.0 / (den >= floor_v ? den : floor_v));
      // change of the prior variance 1/alpha as the stored (float32) alpha has it
      const float a_old = alpha[d];
      const double g_new = 1.0 / (double)a_new, g_old = 1.0 / (double)a_old;
      dg2 += (g_new - g_old) * (g_new - g_old);
      g2 += g_new * g_new;
      if (alpha_prev) alpha_prev[d] = a_old;  // the learned form's features see the step
      alpha[d] = a_new;
      mu[d] = (float)m;
      sdiag[d] = (float)s;
    }
  }
  __shared__ double shm[kMsThreads / 64];
  __shared__ double mine[3], tot[3];
  const double v0 = block_sum(clamped, shm);
  const double v1 = block_sum(dg2, shm);
  const double v2 = block_sum(g2, shm);
  if (threadIdx.x == 0) {
    mine[0] = v0;
    mine[1] = v1;
    mine[2] = v2;
  }
  __syncthreads();
  if (!tree_reduce(parts, cnts, blockIdx.x, gridDim.x, 3, mine, tot)) return;
  finish_mstep(st, tot);
}

hipError_t conv_mstep(const ConvDims& cd, uint64_t seed, int t, const void* X, const double* xm,
                      float* alpha, double alpha_max, float* mu, float* sdiag, const ConvReduce& red, CgScalars* st,
                      hipStream_t s, float* alpha_prev) {
  // conv_update_blocks(cd) blocks: the first column region of the update's
  // reduction workspace (three values per block) serves the M-step's sums
  const unsigned blocks = (unsigned)conv_update_blocks(cd);
  if (cd.fp64)
    hipLaunchKernelGGL(k_conv_mstep<double>, dim3(blocks), dim3(kMsThreads), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t,
                       static_cast<const double*>(X), xm, alpha, alpha_max, mu, sdiag, red.parts, red.cnts, st, alpha_prev);
  else
    hipLaunchKernelGGL(k_conv_mstep<float>, dim3(blocks), dim3(kMsThreads), 0, s, cd.D, cd.ldD, cd.K, cd.perm, cd.nt, seed, t,
                       static_cast<const float*>(X), xm, alpha, alpha_max, mu, sdiag, red.parts, red.cnts, st, alpha_prev);
  return hipGetLastError();
}

// ------------------------------------------------ strided copies between the caller's
// float32 D x K blocks (natural order) and the probe state (float or double,
// leading dimension ldD, element order cd.perm)
template <typename TS, typename TD, bool OUT>
__global__ void k_copy_cols(int64_t D, int K, int perm, const TS* __restrict__ src, int64_t lds,
                            TD* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D * K) return;
  const int64_t k = idx / D, d = idx % D;  // d: state position
  const int64_t n = perm_nat(perm, d);
  if (OUT)
    dst[k * ldd + n] = (TD)src[k * lds + d];
  else
    dst[k * ldd + d] = (TD)src[k * lds + n];
}

hipError_t conv_probes_out(const ConvDims& cd, const void* X, float* out, hipStream_t s) {
  const int64_t tot = cd.D * cd.K;
  const dim3 grid((unsigned)((tot + 255) / 256));
  if (cd.fp64)
    hipLaunchKernelGGL((k_copy_cols<double, float, true>), grid, dim3(256), 0, s, cd.D, cd.K, cd.perm,
                       static_cast<const double*>(X), cd.ldD, out, cd.D);
  else
    hipLaunchKernelGGL((k_copy_cols<float, float, true>), grid, dim3(256), 0, s, cd.D, cd.K, cd.perm,
                       static_cast<const float*>(X), cd.ldD, out, cd.D);
  return hipGetLastError();
}

hipError_t conv_probes_in(const ConvDims& cd, const float* in, void* X, hipStream_t s) {
  const int64_t tot = cd.D * cd.K;
  const dim3 grid((unsigned)((tot + 255) / 256));
  if (cd.fp64)
    hipLaunchKernelGGL((k_copy_cols<float, double, false>), grid, dim3(256), 0, s, cd.D, cd.K, cd.perm, in, cd.D,
                       static_cast<double*>(X), cd.ldD);
  else
    hipLaunchKernelGGL((k_copy_cols<float, float, false>), grid, dim3(256), 0, s, cd.D, cd.K, cd.perm, in, cd.D,
                       static_cast<float*>(X), cd.ldD);
  return hipGetLastError();
}

// single vectors between the state order and the natural order
template <typename T, bool OUT>
__global__ void k_perm_vec(int64_t D, int perm, const T* __restrict__ src, T* __restrict__ dst) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  const int64_t n = perm_nat(perm, d);
  if (OUT)
    dst[n] = src[d];
  else
    dst[d] = src[n];
}

template <typename T, bool OUT>
static hipError_t perm_vec(const ConvDims& cd, const T* src, T* dst, hipStream_t s) {
  if (cd.D == 0) return hipSuccess;
  hipLaunchKernelGGL((k_perm_vec<T, OUT>), dim3((unsigned)((cd.D + 255) / 256)), dim3(256), 0, s, cd.D, cd.perm,
                     src, dst);
  return hipGetLastError();
}
hipError_t perm_out_f32(const ConvDims& cd, const float* src, float* dst, hipStream_t s) {
  return perm_vec<float, true>(cd, src, dst, s);
}
hipError_t perm_in_f32(const ConvDims& cd, const float* src, float* dst, hipStream_t s) {
  return perm_vec<float, false>(cd, src, dst, s);
}
hipError_t perm_out_f64(const ConvDims& cd, const double* src, double* dst, hipStream_t s) {
  return perm_vec<double, true>(cd, src, dst, s);
}
hipError_t perm_in_f64(const ConvDims& cd, const double* src, double* dst, hipStream_t s) {
  return perm_vec<double, false>(cd, src, dst, s);
}

// ------------------------------------------------ probes for tests; fills
__global__ void k_probe_signs(uint64_t seed, int t, int K, int64_t D, float* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D * K) return;
  const int64_t k = idx / D, d = idx % D;
  out[idx] = probe_sign(seed, (uint32_t)t, (uint32_t)k, (uint64_t)d);
}

hipError_t probe_signs_colmajor(uint64_t seed, int t, int K, int64_t D, float* out, hipStream_t s) {
  const int64_t tot = D * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe_signs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, seed, t, K,
                     D, out);
  return hipGetLastError();
}

__global__ void k_fill_f32(float* __restrict__ p, float v, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) p[idx] = v;
}

hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace cofem
