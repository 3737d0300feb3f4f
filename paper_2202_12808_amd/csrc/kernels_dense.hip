// Dense-dictionary kernels of the CoFEM E-step (Sec. 3.1-3.2 of arXiv 2202.12808).
//
// Per CG iteration the operator A P = beta Phi^T (Phi P) + alpha (.) P is applied
// to all K+1 columns at once (mat-vecs replaced by mat-mats, Sec. 3.2) as two
// skinny GEMMs on the matrix cores with v_mfma_f32_32x32x2f32:
//   pass 1  W = Phi P          32-row tiles of Phi,
//   pass 2  Q = Phi^T W + ...  32-coordinate tiles,
// one workgroup of 8 waves per (tile, split); the waves take the split's
// 8-wide reduction groups round-robin and sum their tiles in LDS, and when a
// pass has too few tiles to cover the GPU the reduction is also split across
// workgroups (the last one adds the partials in split order).  The 32 probe
// slots are one MFMA N-tile.  The mean column (column K of Eq. 7) rides along
// on the vector ALU in float64 -- one FMA per Phi element already in registers
// -- so it costs no extra Phi traffic.
//
// Layouts (all owned by the library):
//  * phiA / phiB: Phi and Phi^T cut into 32-row tiles and 8-wide groups; each
//    (tile, group) is one contiguous 1 KiB chunk holding the A operand of four
//    consecutive MFMAs (see k_pack_a32 / k_pack_b32).
//  * probe-column state X, R, P, Q and W: blocked-4 (see DenseDims): the
//    float4 at ((k/4) * 32 + c) is the B fragment of lane (c, (k%8)/4), and
//    the C result's rows 8k' + 4h .. +3 of column c form one float4.
//  * mean-column state: float64 vectors.
#include "cofem_internal.h"

namespace cofem {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// --------------------------------------------------------------- packing
// phiA chunk (t, g), t = 32-row tile, g = 8-column group, at (t * G + g) * 64:
// lane l holds Phi[32 t + l%32][8 g + 4 (l/32) + s], s = 0..3.
__global__ void k_pack_a32(const float* __restrict__ phi, int64_t ld, int64_t N, int64_t D,
                           int64_t G, int64_t tiles, float4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tiles * G * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int64_t g = rest % G, t = rest / G;
  const int64_t n = 32 * t + (lane & 31);
  const int64_t d0 = 8 * g + 4 * (lane >> 5);
  float v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = (n < N && d0 + s < D) ? phi[n * ld + d0 + s] : 0.0f;
  out[idx] = make_float4(v[0], v[1], v[2], v[3]);
}

// phiB chunk (t, g), t = 32-coordinate tile, g = 8-row group:
// lane l holds Phi[8 g + 4 (l/32) + s][32 t + l%32], s = 0..3.
__global__ void k_pack_b32(const float* __restrict__ phi, int64_t ld, int64_t N, int64_t D,
                           int64_t G2, int64_t tiles, float4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tiles * G2 * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int64_t g = rest % G2, t = rest / G2;
  const int64_t d = 32 * t + (lane & 31);
  const int64_t n0 = 8 * g + 4 * (lane >> 5);
  float v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = (n0 + s < N && d < D) ? phi[(n0 + s) * ld + d] : 0.0f;
  out[idx] = make_float4(v[0], v[1], v[2], v[3]);
}

hipError_t dense_pack(const float* phi, int64_t ld, const DenseDims& dd, float* phiA, float* phiB,
                      hipStream_t s) {
  const int64_t G = dd.Dp / 8, tilesA = dd.Np / 32;
  const int64_t totA = tilesA * G * 64;
  hipLaunchKernelGGL(k_pack_a32, dim3((unsigned)((totA + 255) / 256)), dim3(256), 0, s, phi, ld, dd.N,
                     dd.D, G, tilesA, reinterpret_cast<float4*>(phiA));
  const int64_t G2 = dd.Np / 8, tilesB = dd.Dp / 32;
  const int64_t totB = tilesB * G2 * 64;
  hipLaunchKernelGGL(k_pack_b32, dim3((unsigned)((totB + 255) / 256)), dim3(256), 0, s, phi, ld, dd.N,
                     dd.D, G2, tilesB, reinterpret_cast<float4*>(phiB));
  return hipGetLastError();
}

// ------------------------------------------------- b0 = beta Phi^T y (Eq. 5)
// (the dictionary as the problem defines it: float32, or its bfloat16 rounding)
__global__ void k_dense_b0(const void* __restrict__ phi, int kind, int64_t ld, const float* __restrict__ y,
                           double beta, int64_t N, int64_t D, int64_t Dp, double* __restrict__ b0) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= Dp) return;
  double acc = 0.0;
  if (d < D)
    for (int64_t n = 0; n < N; ++n) acc = fma((double)dict_value(phi, kind, n * ld + d), (double)y[n], acc);
  b0[d] = beta * acc;
}

hipError_t dense_b0(const void* phi, int kind, int64_t ld, const float* y, double beta, const DenseDims& dd,
                    double* b0, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_b0, dim3((unsigned)((dd.Dp + 255) / 256)), dim3(256), 0, s, phi, kind, ld, y,
                     beta, dd.N, dd.D, dd.Dp, b0);
  return hipGetLastError();
}

// Blocks of 256 threads for the vector kernels: enough that each thread has
// kVecChunks float4 chunks of the probe block, so the update's loads go out in
// one round (a second dependent round costs a full memory latency).
constexpr int kVecChunks = 1;
int dense_update_blocks(const DenseDims& dd) {
  const int64_t want = (dd.Dp * 8 + kVecChunks * 256 - 1) / (kVecChunks * 256);
  return (int)(want < 1 ? 1 : (want > 1024 ? 1024 : want));
}

// ------------------------------------------------ initial residual R = P = B (Eq. 7)
// (nt mean columns at stride Dp: task j's b0, x, r, p at + j Dp).  With a
// Jacobi diagonal minv: P = Z = M^-1 R and the sums r^T z, r^T r, b^T b
// (= r^T r) per column for finish_init_pcg.
__device__ __forceinline__ void dense_init_body(int64_t blk, int64_t nblk, int64_t D, int64_t Dp, uint64_t seed, int t,
                                                    int K, const double* __restrict__ b0,
                                                    float* __restrict__ X, float* __restrict__ R,
                                                    float* __restrict__ P, double* __restrict__ xm,
                                                    double* __restrict__ rm,
                                                    double* __restrict__ pm,
                                                    double* __restrict__ parts, uint32_t* cnts,
                                                    CgScalars* st, int nt = 1, const float* __restrict__ minv = nullptr) {
  const int64_t gtid = (int64_t)blk * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)nblk * blockDim.x;
  const int c = threadIdx.x & 31;
  double acc = 0.0, accz = 0.0;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    const int64_t d0 = (e4 >> 5) * 4;
    float v[4], z[4];
    const float4 mv = minv ? *reinterpret_cast<const float4*>(minv + d0) : make_float4(1.f, 1.f, 1.f, 1.f);
    const float m4[4] = {mv.x, mv.y, mv.z, mv.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = (d0 + i < D && c < K) ? probe_sign(seed, (uint32_t)t, (uint32_t)c, (uint64_t)(d0 + i)) : 0.0f;
      z[i] = m4[i] * v[i];
      acc += (double)v[i] * (double)v[i];
      accz += (double)v[i] * (double)z[i];
    }
    const float4 r = make_float4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<float4*>(R)[e4] = r;
    reinterpret_cast<float4*>(P)[e4] = make_float4(z[0], z[1], z[2], z[3]);
    reinterpret_cast<float4*>(X)[e4] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  double accm[kMaxDenseTasks] = {0.0, 0.0, 0.0, 0.0}, accmz[kMaxDenseTasks] = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < nt; ++j)
    for (int64_t d = gtid; d < Dp; d += gstride) {
      const double b = b0[j * Dp + d];
      const double z = minv ? (double)minv[d] * b : b;
      rm[j * Dp + d] = b;
      pm[j * Dp + d] = z;
      xm[j * Dp + d] = 0.0;
      accm[j] += b * b;
      accmz[j] += b * z;
    }
  constexpr int kN = kDenseKP + kMaxDenseTasks;
  __shared__ double mine[3 * kN], tot[3 * kN];
  const int nc = kDenseKP + nt;
  if (!minv) {
    dense_block_sums(acc, accm, nt, mine);
    if (!tree_reduce(parts, cnts, blk, nblk, nc, mine, tot)) return;
    finish_init(st, tot);
    return;
  }
  dense_block_sums(accz, accmz, nt, mine);
  dense_block_sums(acc, accm, nt, mine + nc);
  if ((int)threadIdx.x < nc) mine[2 * nc + threadIdx.x] = mine[nc + threadIdx.x];
  __syncthreads();
  if (!tree_reduce(parts, cnts, blk, nblk, 3 * nc, mine, tot)) return;
  finish_init_pcg(st, tot, nc);
}

__global__ __launch_bounds__(256) void k_dense_init(int64_t D, int64_t Dp, uint64_t seed, int t,
                                                    int K, const double* __restrict__ b0,
                                                    float* __restrict__ X, float* __restrict__ R,
                                                    float* __restrict__ P, double* __restrict__ xm,
                                                    double* __restrict__ rm,
                                                    double* __restrict__ pm,
                                                    double* __restrict__ parts, uint32_t* cnts,
                                                    CgScalars* st, int nt, const float* __restrict__ minv) {
  dense_init_body(blockIdx.x, gridDim.x, D, Dp, seed, t, K, b0, X, R, P, xm, rm, pm, parts, cnts, st, nt, minv);
}

hipError_t dense_init(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0,
                      float* X, float* R, float* P, double* xm, double* rm, double* pm,
                      double* parts, uint32_t* cnts, CgScalars* st, hipStream_t s, const float* minv) {
  hipLaunchKernelGGL(k_dense_init, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.D, dd.Dp, seed,
                     t, K, b0, X, R, P, xm, rm, pm, parts, cnts, st, dd.nt, minv);
  return hipGetLastError();
}

// ------------------------------------------------ skinny GEMM tile (32 x 32 + mean)
// v_mfma_f32_32x32x2f32: lane l supplies A[l%32][k] and B[k][l%32] with k = l/32.
// Group g (8 reduction indices) is four MFMAs; MFMA s of group g pairs lane
// half h with reduction index 8g + 4h + s, so lane (c, h) needs
//   A: the packed float4 chunk (one 1 KiB coalesced load per wave),
//   B: rows 8g + 4h .. +3 of column c of the blocked-4 operand -- one float4,
//      two contiguous 512-byte halves per wave,
//   mean column: bm[8g + 4h + s], s = 0..3, staged per workgroup in LDS.
// Vector loads complete in order, so the A and B streams share one ring of
// RING outstanding groups; the LDS reads of the mean values do not touch it.

// One 8-wide group: four MFMAs into the probe tile, four float64 FMAs per
// mean column into the lane's share of that column (m[j]: the four values of
// mean column j for the lane's half, from LDS).
template <int NT>
__device__ __forceinline__ void mma_group(const float4& av, const float4& bv, const double4 (&m)[NT],
                                          floatx16& acc, double (&accm)[NT]) {
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, bv.z, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, bv.w, acc, 0, 0, 0);
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    accm[j] = fma((double)av.x, m[j].x, accm[j]);
    accm[j] = fma((double)av.y, m[j].y, accm[j]);
    accm[j] = fma((double)av.z, m[j].z, accm[j]);
    accm[j] = fma((double)av.w, m[j].w, accm[j]);
  }
}

// The workgroup's mean-column operand for groups [g0, g1): staged once in LDS
// (coalesced), read per group with LDS broadcasts -- the LDS counter is
// separate from the vector-memory counter that paces the Phi ring.  With NT
// mean columns (tasks sharing alpha) the stage holds NT columns, so a range
// may span kMaxStageGroups / NT groups.
constexpr int kMaxStageGroups = 512;  // 4096 values, 32 KiB

template <int WAVES, int RING, int NT>
__device__ __forceinline__ void gemm32(const float4* __restrict__ pa, int64_t g0, int64_t g1,
                                       const float4* __restrict__ B4, const double* __restrict__ bm, int64_t ldm,
                                       floatx16& acc, double (&accm)[NT]) {
  __shared__ double4 sm[kMaxStageGroups * 2];  // [column][group][half] -> 4 values
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 31, h = lane >> 5;
  const int64_t span = g1 - g0;
  const int span2 = (int)(2 * span);
  // (host guarantees NT * span <= kMaxStageGroups)
  for (int64_t e = threadIdx.x; e < span2 * NT; e += blockDim.x) {
    const int64_t j = e / span2, k = e - (e / span2) * span2;
    sm[e] = *reinterpret_cast<const double4*>(bm + j * ldm + 8 * g0 + 4 * k);
  }
  __syncthreads();
  const int64_t n = span > wave ? (span - wave + WAVES - 1) / WAVES : 0;  // steps of this wave
  const int64_t gw = g0 + wave;  // group of step i: gw + WAVES * i
  const int smw = 2 * wave + h;  // sm index of step i: smw + 2 WAVES i (+ j span2 for column j)
  const float4* paw = pa + lane;
  auto mean_of = [&](int64_t i, double4 (&m)[NT]) {
#pragma unroll
    for (int j = 0; j < NT; ++j) m[j] = sm[j * span2 + smw + 2 * WAVES * i];
  };
  double4 m[NT];
  if (n < 2 * RING) {  // short range: no ring
    for (int64_t i = 0; i < n; ++i) {
      const int64_t g = gw + (int64_t)WAVES * i;
      mean_of(i, m);
      mma_group<NT>(paw[g * 64], B4[(2 * g + h) * 32 + c], m, acc, accm);
    }
  } else {
    float4 a[RING], b[RING];
    // prologue: unconditional and in slot order, so the loop-header wait
    // counts are the steady-state ones
#pragma unroll
    for (int r = 0; r < RING; ++r) {
      const int64_t g = gw + (int64_t)WAVES * r;
      a[r] = paw[g * 64];
      b[r] = B4[(2 * g + h) * 32 + c];
      __builtin_amdgcn_sched_barrier(0);
    }
    // steady state: each step consumes its slot, then refills the same slot
    // with the group RING steps ahead, so RING - 1 groups stay in flight.
    int64_t i0 = 0;
    for (; i0 + 2 * RING <= n; i0 += RING) {
#pragma unroll
      for (int r = 0; r < RING; ++r) {
        mean_of(i0 + r, m);
        mma_group<NT>(a[r], b[r], m, acc, accm);
        __builtin_amdgcn_sched_barrier(0);
        const int64_t gn = gw + (int64_t)WAVES * (i0 + r + RING);
        a[r] = paw[gn * 64];
        b[r] = B4[(2 * gn + h) * 32 + c];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // drain: RING .. 2 RING - 1 steps remain
#pragma unroll
    for (int r = 0; r < RING; ++r) {
      const int64_t i = i0 + r;
      mean_of(i, m);
      mma_group<NT>(a[r], b[r], m, acc, accm);
      if (i + RING < n) {
        const int64_t gn = gw + (int64_t)WAVES * (i + RING);
        a[r] = paw[gn * 64];
        b[r] = B4[(2 * gn + h) * 32 + c];
      }
    }
#pragma unroll
    for (int r = 0; r < RING; ++r) {
      const int64_t i = i0 + RING + r;
      if (i < n) {
        mean_of(i, m);
        mma_group<NT>(a[r], b[r], m, acc, accm);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) accm[j] += __shfl_xor(accm[j], 32, 64);  // both halves of tile row c
}

// Sums the waves' tiles through LDS.  Thread e < 256 gets tile rows
// 8k + 4h .. +3 of column c (k = e/64, l = e%64, c = l%32, h = l/32) as a
// float4 -- four consecutive coordinates, i.e. one blocked-4 float4; thread
// e < 32 gets the sums of tile row e of every mean column.
template <int WAVES, int NT>
__device__ __forceinline__ void wg_reduce32(const floatx16& acc, const double (&accm)[NT], float4* out,
                                            double (&outm)[NT]) {
  __shared__ float red[WAVES][16][64];
  __shared__ double redm[WAVES][NT][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
  if (lane < 32)
#pragma unroll
    for (int j = 0; j < NT; ++j) redm[wave][j][lane] = accm[j];
  __syncthreads();
  if (threadIdx.x < 256) {
    const int k = threadIdx.x >> 6, l = threadIdx.x & 63;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int w = 0; w < WAVES; ++w)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] += red[w][4 * k + q][l];
    *out = make_float4(v[0], v[1], v[2], v[3]);
  }
  if (threadIdx.x < 32) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) v += redm[w][j][threadIdx.x];
      outm[j] = v;
    }
  }
}

// blocked-4 float4 index of tile rows 8k + 4h .. +3, column c (thread e < 256)
__device__ __forceinline__ int64_t tile_f4(int64_t row0, int e) {
  const int k = e >> 6, l = e & 63;
  return ((row0 + 8 * k + 4 * (l >> 5)) >> 2) * 32 + (l & 31);
}

// Cross-workgroup split of a tile's reduction: the last of `nsplit`
// workgroups sums the stored partials (split order).  False in the others.
// Mean column j's partial of split sp sits at (sp NT + j) rows_total + row.
template <int NT>
__device__ __forceinline__ bool split_reduce32(int nsplit, int split, int64_t row0, int64_t rows_total,
                                               float* __restrict__ part, double* __restrict__ partm,
                                               uint32_t* counter, float4* v, double (&vm)[NT]) {
  if (nsplit == 1) return true;
  const int e = threadIdx.x;
  if (e < 256) {
    float* dst = part + ((int64_t)split * (rows_total / 4) * 32 + tile_f4(row0, e)) * 4;
    store_agent(dst + 0, v->x);
    store_agent(dst + 1, v->y);
    store_agent(dst + 2, v->z);
    store_agent(dst + 3, v->w);
  }
  if (e < 32)
#pragma unroll
    for (int j = 0; j < NT; ++j) store_agent(&partm[((int64_t)split * NT + j) * rows_total + row0 + e], vm[j]);
  if (!last_block_ticket(counter, (uint32_t)nsplit)) return false;
  // partials loaded four splits at a time (16 loads in flight), summed in
  // split order
  if (e < 256) {
    float t[4] = {0.f, 0.f, 0.f, 0.f};
    for (int sp0 = 0; sp0 < nsplit; sp0 += 4) {
      float x[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sp = sp0 + u < nsplit ? sp0 + u : sp0;
        const float* src = part + ((int64_t)sp * (rows_total / 4) * 32 + tile_f4(row0, e)) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) x[u][q] = load_agent(src + q);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (sp0 + u < nsplit)
#pragma unroll
          for (int q = 0; q < 4; ++q) t[q] += x[u][q];
    }
    *v = make_float4(t[0], t[1], t[2], t[3]);
  }
  if (e < 32) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      double t = 0.0;
      for (int sp0 = 0; sp0 < nsplit; sp0 += 4) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int sp = sp0 + u < nsplit ? sp0 + u : sp0;
          x[u] = load_agent(&partm[((int64_t)sp * NT + j) * rows_total + row0 + e]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (sp0 + u < nsplit) t += x[u];
      }
      vm[j] = t;
    }
  }
  if (e == 0) store_agent(counter, 0u);
  return true;
}

constexpr int kGemmWaves = 8;

// ------------------------------------------------ pass 1: W = Phi P
// NT mean columns (tasks sharing alpha): column j of the float64 block at
// pm + j Dp, its product at wm + j Np.
template <int RING, int NT>
__global__ __launch_bounds__(64 * kGemmWaves) void k_dense_pass1(
    const float4* __restrict__ phiA, int64_t G, int64_t gps, int nsplit, int64_t Np, int64_t Dp,
    const float* __restrict__ P, const double* __restrict__ pm, float* __restrict__ Wpart,
    double* __restrict__ wmpart, float* __restrict__ W, double* __restrict__ wm,
    uint32_t* __restrict__ cnts, CgScalars* __restrict__ st, int apply_only) {
  if (!apply_only && st->stop) return;
  const int64_t tile = blockIdx.x;
  const int split = blockIdx.y;
  const int64_t g0 = split * gps;
  const int64_t g1 = (g0 + gps < G) ? g0 + gps : G;
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
  double accm[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) accm[j] = 0.0;
  gemm32<kGemmWaves, RING, NT>(phiA + tile * G * 64, g0, g1, reinterpret_cast<const float4*>(P), pm, Dp, acc,
                               accm);
  float4 v;
  double vm[NT];
  wg_reduce32<kGemmWaves, NT>(acc, accm, &v, vm);
  const int64_t row0 = tile * 32;
  if (!split_reduce32<NT>(nsplit, split, row0, Np, Wpart, wmpart, &cnts[tile * kCounterStride], &v, vm)) return;
  if (threadIdx.x < 256) reinterpret_cast<float4*>(W)[tile_f4(row0, threadIdx.x)] = v;
  if (threadIdx.x < 32)
#pragma unroll
    for (int j = 0; j < NT; ++j) wm[j * Np + row0 + threadIdx.x] = vm[j];
}

hipError_t dense_pass1(const DenseDims& dd, const float* phiA, const float* P, const double* pm,
                       float* Wpart, double* wmpart, float* W, double* wm, uint32_t* cnts,
                       CgScalars* st, int apply_only, hipStream_t s) {
  const int64_t tiles = dd.Np / 32, G = dd.Dp / 8;
  if (!dense_split_ok(G, dd.S1, dd.nt)) return hipErrorInvalidValue;
  const int64_t gps = (G + dd.S1 - 1) / dd.S1;
#define COFEM_PASS1(RG, NT)                                                                               \
  hipLaunchKernelGGL((k_dense_pass1<RG, NT>), dim3((unsigned)tiles, (unsigned)dd.S1), dim3(64 * kGemmWaves), \
                     0, s, reinterpret_cast<const float4*>(phiA), G, gps, dd.S1, dd.Np, dd.Dp, P, pm, Wpart,   \
                     wmpart, W, wm, cnts, st, apply_only)
  if (dd.nt == 1) {
    switch (dd.ring) {
      case 1: COFEM_PASS1(1, 1); break;
      case 2: COFEM_PASS1(2, 1); break;
      case 8: COFEM_PASS1(8, 1); break;
      default: COFEM_PASS1(4, 1); break;
    }
  } else {
    switch (dd.nt) {  // several tasks: the default ring only
      case 2: COFEM_PASS1(4, 2); break;
      case 3: COFEM_PASS1(4, 3); break;
      case 4: COFEM_PASS1(4, 4); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef COFEM_PASS1
  return hipGetLastError();
}

// ------------------------------------------------ pass 2: Q = beta Phi^T W + alpha (.) P
// The epilogue also forms the per-column dots gam = p^T q, del = r^T q and
// eta = q^T q (del and eta weighted by M^-1 when minv is set, so b_c comes
// out as the preconditioned r'^T z' / r^T z); the tree reduction's final
// workgroup turns them into a_c, b_c.
// NT mean columns: column j of W at wm + j Np, of p, r, q at + j Dp.
template <int RING, int NT>
__global__ __launch_bounds__(64 * kGemmWaves) void k_dense_pass2(
    const float4* __restrict__ phiB, int64_t G2, int64_t gps, int nsplit, int64_t Np, int64_t Dp,
    const float* __restrict__ W, const double* __restrict__ wm, const float* __restrict__ P,
    const double* __restrict__ pm, const float* __restrict__ R, const double* __restrict__ rm,
    const float* __restrict__ alpha, double beta, float* __restrict__ Qpart,
    double* __restrict__ qmpart, float* __restrict__ Q, double* __restrict__ qm,
    double* __restrict__ parts, uint32_t* __restrict__ cnts, uint32_t* __restrict__ split_cnts,
    CgScalars* __restrict__ st, int apply_only, const float* __restrict__ minv) {
  if (!apply_only && st->stop) return;
  const CgCtl ctl = load_cg_ctl(st);
  constexpr int nc = kDenseKP + NT;
  const int64_t tile = blockIdx.x;
  const int split = blockIdx.y;
  const int64_t g0 = split * gps;
  const int64_t g1 = (g0 + gps < G2) ? g0 + gps : G2;
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
  double accm[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) accm[j] = 0.0;
  gemm32<kGemmWaves, RING, NT>(phiB + tile * G2 * 64, g0, g1, reinterpret_cast<const float4*>(W), wm, Np, acc,
                               accm);
  float4 v;
  double vm[NT];
  wg_reduce32<kGemmWaves, NT>(acc, accm, &v, vm);
  const int64_t d0 = tile * 32;
  if (!split_reduce32<NT>(nsplit, split, d0, Dp, Qpart, qmpart, &split_cnts[tile * kCounterStride], &v, vm))
    return;

  __shared__ double sdots[3][256];
  __shared__ double mine[3 * nc], tot[3 * nc];
  const int e = threadIdx.x;
  if (e < 256) {
    const int64_t i4 = tile_f4(d0, e);
    const int64_t dq = d0 + 8 * (e >> 6) + 4 * ((e & 63) >> 5);  // first of four coordinates
    const float4 p = reinterpret_cast<const float4*>(P)[i4];
    const float4 al = *reinterpret_cast<const float4*>(alpha + dq);
    const float bf = (float)beta;
    float4 q;
    q.x = fmaf(al.x, p.x, bf * v.x);
    q.y = fmaf(al.y, p.y, bf * v.y);
    q.z = fmaf(al.z, p.z, bf * v.z);
    q.w = fmaf(al.w, p.w, bf * v.w);
    reinterpret_cast<float4*>(Q)[i4] = q;
    if (!apply_only) {
      const float4 r = reinterpret_cast<const float4*>(R)[i4];
      sdots[0][e] = (double)p.x * q.x + (double)p.y * q.y + (double)p.z * q.z + (double)p.w * q.w;
      float4 mq = q;  // M^-1 q
      if (minv) {
        const float4 mv = *reinterpret_cast<const float4*>(minv + dq);
        mq = make_float4(mv.x * q.x, mv.y * q.y, mv.z * q.z, mv.w * q.w);
      }
      sdots[1][e] = (double)r.x * mq.x + (double)r.y * mq.y + (double)r.z * mq.z + (double)r.w * mq.w;
      sdots[2][e] = (double)q.x * mq.x + (double)q.y * mq.y + (double)q.z * mq.z + (double)q.w * mq.w;
    }
  }
  double gmm[NT], dmm[NT], emm[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) gmm[j] = dmm[j] = emm[j] = 0.0;
  if (e < 32) {
    const int64_t d = d0 + e;
    const double a = (double)alpha[d];
    const double mvd = minv ? (double)minv[d] : 1.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const double p = pm[j * Dp + d];
      const double q = beta * vm[j] + a * p;
      qm[j * Dp + d] = q;
      gmm[j] = p * q;
      dmm[j] = rm[j * Dp + d] * (mvd * q);
      emm[j] = q * (mvd * q);
    }
  }
  if (apply_only) return;
  if (e < 64) {  // wave 0: mean-column dots over the tile's 32 coordinates
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      for (int off = 16; off > 0; off >>= 1) {
        gmm[j] += __shfl_xor(gmm[j], off, 64);
        dmm[j] += __shfl_xor(dmm[j], off, 64);
        emm[j] += __shfl_xor(emm[j], off, 64);
      }
      if (e == 0) {
        mine[kDenseKP + j] = gmm[j];
        mine[nc + kDenseKP + j] = dmm[j];
        mine[2 * nc + kDenseKP + j] = emm[j];
      }
    }
  }
  __syncthreads();
  if (e < 3 * kDenseKP) {  // column c's 8 entries: e' = 64k + 32h + c
    const int kind = e / kDenseKP, cc = e % kDenseKP;
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sacc += sdots[kind][64 * (q >> 1) + 32 * (q & 1) + cc];
    mine[kind * nc + cc] = sacc;
  }
  __syncthreads();
  if (!tree_reduce(parts, cnts, tile, gridDim.x, 3 * nc, mine, tot)) return;
  finish_step(st, tot, ctl);
}

hipError_t dense_pass2(const DenseDims& dd, const float* phiB, const float* W, const double* wm,
                       const float* P, const double* pm, const float* R, const double* rm,
                       const float* alpha, double beta, float* Qpart, double* qmpart, float* Q,
                       double* qm, double* gpart, uint32_t* counter, uint32_t* split_cnts,
                       CgScalars* st, int apply_only, hipStream_t s, const float* minv) {
  const int64_t tiles = dd.Dp / 32, G2 = dd.Np / 8;
  if (!dense_split_ok(G2, dd.S2, dd.nt)) return hipErrorInvalidValue;
  const int64_t gps = (G2 + dd.S2 - 1) / dd.S2;
#define COFEM_PASS2(RG, NT)                                                                               \
  hipLaunchKernelGGL((k_dense_pass2<RG, NT>), dim3((unsigned)tiles, (unsigned)dd.S2), dim3(64 * kGemmWaves), \
                     0, s, reinterpret_cast<const float4*>(phiB), G2, gps, dd.S2, dd.Np, dd.Dp, W, wm, P, pm, R, \
                     rm, alpha, beta, Qpart, qmpart, Q, qm, gpart, counter, split_cnts, st, apply_only, minv)
  if (dd.nt == 1) {
    switch (dd.ring) {
      case 1: COFEM_PASS2(1, 1); break;
      case 2: COFEM_PASS2(2, 1); break;
      case 8: COFEM_PASS2(8, 1); break;
      default: COFEM_PASS2(4, 1); break;
    }
  } else {
    switch (dd.nt) {
      case 2: COFEM_PASS2(4, 2); break;
      case 3: COFEM_PASS2(4, 3); break;
      case 4: COFEM_PASS2(4, 4); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef COFEM_PASS2
  return hipGetLastError();
}

// Splits of a pass's reduction over workgroups: about two resident
// 512-thread workgroups per CU (512 in all), at least 32 groups per wave.
// Measured on the 4096 x 16384 problem, 1024 workgroups (more splits, more
// partial-sum traffic) was no faster than 512.
int dense_split(int64_t tiles, int64_t groups, int nt) {
  int64_t s = (512 + tiles - 1) / tiles;
  const int64_t most = groups / (32 * kGemmWaves);
  if (s > most) s = most;
  if (s > 16) s = 16;
  const int64_t stage = kMaxStageGroups / nt;  // LDS staging limit (nt mean columns)
  const int64_t least = (groups + stage - 1) / stage;
  if (s < least) s = least;
  return (int)(s < 1 ? 1 : s);
}

bool dense_split_ok(int64_t groups, int splits, int nt) {
  return splits >= 1 && nt >= 1 && (groups + splits - 1) / splits <= kMaxStageGroups / nt;
}

// ------------------------------------------------ CG update
// x += a p ; r -= a q ; p <- r + b p ; rho' = ||r||^2 and the stop test.
// With a Jacobi diagonal minv: z = M^-1 r, p <- z + b p, and the sums r^T z
// (rho') and r^T r (the stop test) per column for finish_update_pcg.
__device__ __forceinline__ void dense_update_body(int64_t blk, int64_t nblk, int64_t Dp, float* __restrict__ X,
                                                      float* __restrict__ R, float* __restrict__ P,
                                                      const float* __restrict__ Q,
                                                      double* __restrict__ xm,
                                                      double* __restrict__ rm,
                                                      double* __restrict__ pm,
                                                      const double* __restrict__ qm,
                                                      double* __restrict__ parts, uint32_t* cnts,
                                                      CgScalars* st, int nt = 1,
                                                      const float* __restrict__ minv = nullptr) {
  const int64_t gtid = (int64_t)blk * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)nblk * blockDim.x;
  const int c = threadIdx.x & 31;
  const int64_t n4 = Dp * 8;
  // Elements go two per round, both rounds' loads issued before any use.  The
  // first round's state is loaded together with the scalars and the stop flag
  // (all in bounds), so the flag's latency hides under the data's; the flag
  // only decides whether anything is written.
  float4 x[2], r[2], p[2], q[2];
  auto load2 = [&](int64_t e4) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t e = e4 + u * gstride;
      if (e < n4) {
        x[u] = reinterpret_cast<float4*>(X)[e];
        r[u] = reinterpret_cast<float4*>(R)[e];
        p[u] = reinterpret_cast<float4*>(P)[e];
        q[u] = reinterpret_cast<const float4*>(Q)[e];
      }
    }
  };
  load2(gtid);
  // this thread's first element of the float64 mean column, in the same round
  double m_x = 0.0, m_r = 0.0, m_p = 0.0, m_q = 0.0;
  if (gtid < Dp) {
    m_x = xm[gtid];
    m_r = rm[gtid];
    m_p = pm[gtid];
    m_q = qm[gtid];
  }
  const CgCtl ctl = load_cg_ctl(st);
  const int stop = st->stop;
  const float a = (float)st->a[c], b = (float)st->b[c];
  const double am = st->a[kDenseKP], bmm = st->b[kDenseKP];
  if (stop) return;
  double acc = 0.0, accz = 0.0;
  for (int64_t e4 = gtid; e4 < n4; e4 += 2 * gstride) {
    if (e4 != gtid) load2(e4);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t e = e4 + u * gstride;
      if (e < n4) {
        float4 xv = x[u], rv = r[u], pv = p[u];
        const float4 qv = q[u];
        xv.x = fmaf(a, pv.x, xv.x);
        xv.y = fmaf(a, pv.y, xv.y);
        xv.z = fmaf(a, pv.z, xv.z);
        xv.w = fmaf(a, pv.w, xv.w);
        rv.x = fmaf(-a, qv.x, rv.x);
        rv.y = fmaf(-a, qv.y, rv.y);
        rv.z = fmaf(-a, qv.z, rv.z);
        rv.w = fmaf(-a, qv.w, rv.w);
        float4 zv = rv;
        if (minv) {  // e's four coordinates start at (e >> 5) * 4
          const float4 mv = *reinterpret_cast<const float4*>(minv + (e >> 5) * 4);
          zv = make_float4(mv.x * rv.x, mv.y * rv.y, mv.z * rv.z, mv.w * rv.w);
          accz += (double)rv.x * zv.x + (double)rv.y * zv.y + (double)rv.z * zv.z + (double)rv.w * zv.w;
        }
        pv.x = fmaf(b, pv.x, zv.x);
        pv.y = fmaf(b, pv.y, zv.y);
        pv.z = fmaf(b, pv.z, zv.z);
        pv.w = fmaf(b, pv.w, zv.w);
        reinterpret_cast<float4*>(X)[e] = xv;
        reinterpret_cast<float4*>(R)[e] = rv;
        reinterpret_cast<float4*>(P)[e] = pv;
        acc += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z + (double)rv.w * rv.w;
      }
    }
  }
  double accm[kMaxDenseTasks] = {0.0, 0.0, 0.0, 0.0}, accmz[kMaxDenseTasks] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t d = gtid; d < Dp; d += gstride) {
    if (d != gtid) {
      m_x = xm[d];
      m_r = rm[d];
      m_p = pm[d];
      m_q = qm[d];
    }
    xm[d] = fma(am, m_p, m_x);
    const double rv = fma(-am, m_q, m_r);
    const double zv = minv ? (double)minv[d] * rv : rv;
    rm[d] = rv;
    pm[d] = fma(bmm, m_p, zv);
    accm[0] += rv * rv;
    accmz[0] += rv * zv;
  }
  // further mean columns (tasks sharing alpha)
  for (int j = 1; j < nt; ++j) {
    const double aj = st->a[kDenseKP + j], bj = st->b[kDenseKP + j];
    const int64_t o = j * Dp;
    for (int64_t d = gtid; d < Dp; d += gstride) {
      const double xv = xm[o + d], rv0 = rm[o + d], pv = pm[o + d], qv = qm[o + d];
      xm[o + d] = fma(aj, pv, xv);
      const double rv = fma(-aj, qv, rv0);
      const double zv = minv ? (double)minv[d] * rv : rv;
      rm[o + d] = rv;
      pm[o + d] = fma(bj, pv, zv);
      accm[j] += rv * rv;
      accmz[j] += rv * zv;
    }
  }
  constexpr int kN = kDenseKP + kMaxDenseTasks;
  __shared__ double mine[2 * kN], tot[2 * kN];
  const int nc = kDenseKP + nt;
  if (!minv) {
    dense_block_sums(acc, accm, nt, mine);
    if (!tree_reduce(parts, cnts, blk, nblk, nc, mine, tot)) return;
    finish_update(st, tot, ctl);
    return;
  }
  dense_block_sums(accz, accmz, nt, mine);
  dense_block_sums(acc, accm, nt, mine + nc);
  if (!tree_reduce(parts, cnts, blk, nblk, 2 * nc, mine, tot)) return;
  finish_update_pcg(st, tot, nc, ctl);
}

__global__ __launch_bounds__(256) void k_dense_update(int64_t Dp, float* __restrict__ X,
                                                      float* __restrict__ R, float* __restrict__ P,
                                                      const float* __restrict__ Q,
                                                      double* __restrict__ xm,
                                                      double* __restrict__ rm,
                                                      double* __restrict__ pm,
                                                      const double* __restrict__ qm,
                                                      double* __restrict__ parts, uint32_t* cnts,
                                                      CgScalars* st, int nt, const float* __restrict__ minv) {
  dense_update_body(blockIdx.x, gridDim.x, Dp, X, R, P, Q, xm, rm, pm, qm, parts, cnts, st, nt, minv);
}

hipError_t dense_update(const DenseDims& dd, float* X, float* R, float* P, const float* Q,
                        double* xm, double* rm, double* pm, const double* qm, double* parts,
                        uint32_t* cnts, CgScalars* st, hipStream_t s, const float* minv) {
  hipLaunchKernelGGL(k_dense_update, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.Dp, X, R, P,
                     Q, xm, rm, pm, qm, parts, cnts, st, dd.nt, minv);
  return hipGetLastError();
}

// ------------------------------------------------ Jacobi diagonal (Sec. 3.2 solver, not in the paper)
// cn_d = ||Phi e_d||^2 = sum_n Phi[n][d]^2 (float64 sums; one thread per
// column d, so a row's entries are read by consecutive threads), zero for the
// padding columns.
__global__ void k_dense_colnorm(const void* __restrict__ phi, int kind, int64_t ld, int64_t N, int64_t D, int64_t Dp,
                                float* __restrict__ cn) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= Dp) return;
  double acc = 0.0;
  if (d < D)
    for (int64_t n = 0; n < N; ++n) {
      const double v = (double)dict_value(phi, kind, n * ld + d);
      acc += v * v;
    }
  cn[d] = (float)acc;
}

hipError_t dense_colnorms(const void* phi, int dict_kind, int64_t ld, const DenseDims& dd, float* cn,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_dense_colnorm, dim3((unsigned)((dd.Dp + 255) / 256)), dim3(256), 0, s, phi, dict_kind, ld,
                     dd.N, dd.D, dd.Dp, cn);
  return hipGetLastError();
}

// M^-1 = 1 / diag(A) = 1 / (beta ||Phi e_d||^2 + alpha_d) for d < D; zero in
// the padding, whose state stays zero.
__global__ void k_dense_jacobi(int64_t D, int64_t Dp, const float* __restrict__ cn, double beta,
                               const float* __restrict__ alpha, float* __restrict__ minv) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= Dp) return;
  minv[d] = d < D ? (float)(1.0 / (beta * (double)cn[d] + (double)alpha[d])) : 0.0f;
}

hipError_t dense_jacobi(const DenseDims& dd, const float* cn, double beta, const float* alpha, float* minv,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_dense_jacobi, dim3((unsigned)((dd.Dp + 255) / 256)), dim3(256), 0, s, dd.D, dd.Dp, cn, beta,
                     alpha, minv);
  return hipGetLastError();
}

// ------------------------------------------------ true residual (final check of a solve)
// ||b_c - q_c||^2 per column, float64 sums, with q = A x from the operator
// passes applied to X and B regenerated: probes of EM iteration t (Eq. 7) in
// rows d < D, zero in the padding rows, and b0 for the mean column.
__global__ __launch_bounds__(256) void k_dense_true_resid(int64_t D, int64_t Dp, uint64_t seed, int t, int K,
                                                          const double* __restrict__ b0,
                                                          const float* __restrict__ Q,
                                                          const double* __restrict__ qm,
                                                          double* __restrict__ parts, uint32_t* cnts,
                                                          CgScalars* st, int nt) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  const int c = threadIdx.x & 31;  // gstride is a multiple of 32: fixed column per thread
  double acc = 0.0;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    const float4 q = reinterpret_cast<const float4*>(Q)[e4];
    const int64_t d0 = (e4 >> 5) * 4;
    const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t d = d0 + i;
      const double b = (c < K && d < D) ? (double)probe_sign(seed, (uint32_t)t, (uint32_t)c, (uint64_t)d) : 0.0;
      const double e = b - (double)qv[i];
      acc += e * e;
    }
  }
  double accm[kMaxDenseTasks] = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < nt; ++j)
    for (int64_t d = gtid; d < Dp; d += gstride) {
      const double e = b0[j * Dp + d] - qm[j * Dp + d];
      accm[j] += e * e;
    }
  __shared__ double mine[kDenseKP + kMaxDenseTasks], tot[kDenseKP + kMaxDenseTasks];
  dense_block_sums(acc, accm, nt, mine);
  if (!tree_reduce(parts, cnts, blockIdx.x, gridDim.x, kDenseKP + nt, mine, tot)) return;
  finish_true_resid(st, tot);
}

hipError_t dense_true_resid(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0,
                            const float* Q, const double* qm, double* parts, uint32_t* cnts,
                            CgScalars* st, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_true_resid, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.D, dd.Dp, seed,
                     t, K, b0, Q, qm, parts, cnts, st, dd.nt);
  return hipGetLastError();
}

// ------------------------------------------------ diagonal estimate + M-step (Eq. 6, Eq. 8)
__device__ __forceinline__ void dense_mstep_body(int64_t blk, int64_t nblk, int64_t D, uint64_t seed, int t, int K,
                                                     const float* __restrict__ X,
                                                     const double* __restrict__ xm,
                                                     float* __restrict__ alpha, double alpha_max,
                                                     float* __restrict__ mu,
                                                     float* __restrict__ sdiag, double* parts, uint32_t* cnts,
                                                     CgScalars* st, int nt = 1, int64_t ldm = 0) {
  const int64_t gtid = (int64_t)blk * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)nblk * blockDim.x;
  const double floor_v = 1.0 / alpha_max;
  double clamped = 0.0, dg2 = 0.0, g2 = 0.0;
  for (int64_t d = gtid; d < D; d += gstride) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k)
      acc += (double)probe_sign(seed, (uint32_t)t, (uint32_t)k, (uint64_t)d) * (double)X[blk4(d, k)];
    const double s = acc / (double)K;
    const double m = xm[d];
    // tasks sharing alpha: the mean of their squared means
    double m2 = m * m;
    if (nt > 1) {
      for (int j = 1; j < nt; ++j) {
        const double mj = xm[j * ldm + d];
        m2 += mj * mj;
      }
      m2 /= (double)nt;
    }
    const double den = m2 + s;
    if (!(den >= floor_v)) clamped += 1.0;
    const float a_new = (float)(1.0 / (den >= floor_v ? den : floor_v));
    // change of the prior variance 1/alpha as the stored (float32) alpha has it
    const double g_new = 1.0 / (double)a_new, g_old = 1.0 / (double)alpha[d];
    dg2 += (g_new - g_old) * (g_new - g_old);
    g2 += g_new * g_new;
    alpha[d] = a_new;
    mu[d] = (float)m;
    sdiag[d] = (float)s;
  }
  __shared__ double shm[8];
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
  if (!tree_reduce(parts, cnts, blk, nblk, 3, mine, tot)) return;
  finish_mstep(st, tot);
}

__global__ __launch_bounds__(256) void k_dense_mstep(int64_t D, uint64_t seed, int t, int K,
                                                     const float* __restrict__ X,
                                                     const double* __restrict__ xm,
                                                     float* __restrict__ alpha, double alpha_max,
                                                     float* __restrict__ mu,
                                                     float* __restrict__ sdiag, double* parts, uint32_t* cnts,
                                                     CgScalars* st, int nt, int64_t ldm) {
  dense_mstep_body(blockIdx.x, gridDim.x, D, seed, t, K, X, xm, alpha, alpha_max, mu, sdiag, parts, cnts, st, nt,
                   ldm);
}

hipError_t dense_mstep(const DenseDims& dd, uint64_t seed, int t, int K, const float* X,
                       const double* xm, float* alpha, double alpha_max, float* mu, float* sdiag,
                       double* parts, uint32_t* cnts, CgScalars* st, hipStream_t s) {
  // at most dense_update_blocks(dd) blocks: the update's reduction tree
  // (parts, cnts) serves the M-step's sums
  const int64_t want = (dd.D + 255) / 256, cap = dense_update_blocks(dd);
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
  hipLaunchKernelGGL(k_dense_mstep, dim3(blocks), dim3(256), 0, s, dd.D, seed, t, K, X, xm, alpha,
                     alpha_max, mu, sdiag, parts, cnts, st, dd.nt, dd.Dp);
  return hipGetLastError();
}

// ------------------------------------------------ layout conversions (tests, hooks)
__global__ void k_blk4_to_col(int64_t D, int K, const float* __restrict__ Xb, float* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D * K) return;
  const int64_t k = idx / D, d = idx % D;
  out[idx] = Xb[blk4(d, (int)k)];
}

__global__ void k_col_to_blk4(int64_t D, int64_t Dp, int K, const float* __restrict__ in,
                              float* __restrict__ Xb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Dp * kDenseKP) return;
  const int64_t d = (idx >> 7) * 4 + (idx & 3);
  const int c = (int)((idx >> 2) & 31);
  Xb[idx] = (d < D && c < K) ? in[(int64_t)c * D + d] : 0.0f;
}

hipError_t dense_to_colmajor(const DenseDims& dd, int K, const float* Xb, float* out, hipStream_t s) {
  const int64_t tot = dd.D * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_blk4_to_col, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dd.D, K, Xb,
                     out);
  return hipGetLastError();
}

hipError_t dense_from_colmajor(const DenseDims& dd, int K, const float* in, float* Xb, hipStream_t s) {
  const int64_t tot = dd.Dp * kDenseKP;
  hipLaunchKernelGGL(k_col_to_blk4, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dd.D, dd.Dp,
                     K, in, Xb);
  return hipGetLastError();
}

}  // namespace cofem

namespace cofem {

// ------------------------------------------------ batched form: grouped vector kernels
// Work item a = block index within the problem (p.nvec blocks per problem).
__global__ __launch_bounds__(256) void k_batch_init(const BatchItem* __restrict__ items,
                                                    const BatchProblem* __restrict__ probs, int t, int K) {
  const BatchItem it = items[blockIdx.x];
  const BatchProblem& p = probs[it.prob];
  dense_init_body(it.a, p.nvec, p.D, p.Dp, p.seed, t, K, p.b0, p.X, p.R, p.P, p.xm, p.rm, p.pm, p.parts_init,
                  p.cnts_init, p.st);
}

__global__ __launch_bounds__(256) void k_batch_update(const BatchItem* __restrict__ items,
                                                      const BatchProblem* __restrict__ probs) {
  const BatchItem it = items[blockIdx.x];
  const BatchProblem& p = probs[it.prob];
  dense_update_body(it.a, p.nvec, p.Dp, p.X, p.R, p.P, p.Q, p.xm, p.rm, p.pm, p.qm, p.parts_upd, p.cnts_upd, p.st);
}

__global__ __launch_bounds__(256) void k_batch_mstep(const BatchItem* __restrict__ items,
                                                     const BatchProblem* __restrict__ probs, int t, int K,
                                                     double alpha_max) {
  const BatchItem it = items[blockIdx.x];
  const BatchProblem& p = probs[it.prob];
  dense_mstep_body(it.a, p.nvec, p.D, p.seed, t, K, p.X, p.xm, p.alpha, alpha_max, p.mu, p.sdiag, p.parts_upd,
                   p.cnts_upd, p.st);
}

// Number of problems whose solve has not stopped (one block).
__global__ __launch_bounds__(256) void k_batch_running(const BatchProblem* __restrict__ probs, int n,
                                                       int32_t* __restrict__ out) {
  __shared__ double shm[8];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += probs[i].st->stop ? 0.0 : 1.0;
  const double tot = block_sum(v, shm);
  if (threadIdx.x == 0) out[0] = (int32_t)tot;
}

hipError_t batch_init(const BatchItem* items, int n, const BatchProblem* probs, int t, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3((unsigned)n), dim3(256), 0, s, items, probs, t, K);
  return hipGetLastError();
}

hipError_t batch_update(const BatchItem* items, int n, const BatchProblem* probs, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_update, dim3((unsigned)n), dim3(256), 0, s, items, probs);
  return hipGetLastError();
}

hipError_t batch_mstep(const BatchItem* items, int n, const BatchProblem* probs, int t, int K, double alpha_max,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_batch_mstep, dim3((unsigned)n), dim3(256), 0, s, items, probs, t, K, alpha_max);
  return hipGetLastError();
}

hipError_t batch_running(const BatchProblem* probs, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_running, dim3(1), dim3(256), 0, s, probs, n, out);
  return hipGetLastError();
}

}  // namespace cofem
