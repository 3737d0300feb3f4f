// Low-precision dictionary kernels of the mixed-precision form of the dense
// E-step: Phi rounded once to bfloat16 drives the inner CG solves of an
// iterative refinement whose outer residual B - A X uses the float32 Phi
// (the passes of kernels_dense.hip) with float64 sums.
//
// Per inner CG iteration the two passes run on v_mfma_f32_32x32x16_bf16:
//   pass 1  W = Phi~ P,    pass 2  Q = beta Phi~^T W + alpha (.) P  (+ the CG dots).
// The float32 operand block (P, then W) is split in registers into a
// bfloat16 head and a bfloat16 tail (p = hi + lo + O(2^-17 |p|)), so each
// 16-wide group is two MFMAs per tile and the operator stays linear to
// about float32 accuracy: only Phi is rounded.  The float64 mean column rides
// along as float64 FMAs on the bfloat16 values (exact in float64).
//
// Layouts:
//  * phiA16 / phiB16: Phi and Phi^T cut into 32-row tiles and 16-wide groups;
//    chunk (t, g) is 1 KiB, lane l holding the eight bfloat16 of its MFMA A
//    fragment (k_pack_a16 / k_pack_b16).  Half the bytes of the float32 copy.
//  * probe-column state: the blocked-4 float32 layout of kernels_dense.hip,
//    so the update, init and M-step kernels are shared with the float32 path.
// Each workgroup takes two adjacent 32-row tiles, so every operand fragment
// it loads feeds four MFMAs.
#include "cofem_internal.h"

namespace cofem {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float bf16_lo_as_float(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi_as_float(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// --------------------------------------------------------------- packing
// phiA16 chunk (t, g), t = 32-row tile, g = 16-column group, at (t * G + g) * 64
// (uint4 units): lane l holds bf16(Phi[32 t + l%32][16 g + 8 (l/32) + s]),
// s = 0..7, element s in the low (s even) or high half of word s/2.
__global__ void k_pack_a16(const void* __restrict__ phi, int kind, int64_t ld, int64_t N, int64_t D, int64_t G,
                           int64_t tiles, uint4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tiles * G * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int64_t g = rest % G, t = rest / G;
  const int64_t n = 32 * t + (lane & 31);
  const int64_t d0 = 16 * g + 8 * (lane >> 5);
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t d = d0 + 2 * q;
    const uint32_t lo = (n < N && d < D) ? dict_bf16_bits(phi, kind, n * ld + d) : 0u;
    const uint32_t hi = (n < N && d + 1 < D) ? dict_bf16_bits(phi, kind, n * ld + d + 1) : 0u;
    w[q] = lo | (hi << 16);
  }
  out[idx] = make_uint4(w[0], w[1], w[2], w[3]);
}

// phiB16 chunk (t, g), t = 32-coordinate tile, g = 16-row group:
// lane l holds bf16(Phi[16 g + 8 (l/32) + s][32 t + l%32]), s = 0..7.
__global__ void k_pack_b16(const void* __restrict__ phi, int kind, int64_t ld, int64_t N, int64_t D, int64_t G2,
                           int64_t tiles, uint4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tiles * G2 * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int64_t g = rest % G2, t = rest / G2;
  const int64_t d = 32 * t + (lane & 31);
  const int64_t n0 = 16 * g + 8 * (lane >> 5);
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t n = n0 + 2 * q;
    const uint32_t lo = (n < N && d < D) ? dict_bf16_bits(phi, kind, n * ld + d) : 0u;
    const uint32_t hi = (n + 1 < N && d < D) ? dict_bf16_bits(phi, kind, (n + 1) * ld + d) : 0u;
    w[q] = lo | (hi << 16);
  }
  out[idx] = make_uint4(w[0], w[1], w[2], w[3]);
}

hipError_t dense_pack16(const void* phi, int kind, int64_t ld, const DenseDims& dd, void* phiA16, void* phiB16,
                        hipStream_t s) {
  const int64_t G = dd.Dp / 16, tilesA = dd.Np / 32;
  const int64_t totA = tilesA * G * 64;
  hipLaunchKernelGGL(k_pack_a16, dim3((unsigned)((totA + 255) / 256)), dim3(256), 0, s, phi, kind, ld, dd.N, dd.D,
                     G, tilesA, static_cast<uint4*>(phiA16));
  const int64_t G2 = dd.Np / 16, tilesB = dd.Dp / 32;
  const int64_t totB = tilesB * G2 * 64;
  hipLaunchKernelGGL(k_pack_b16, dim3((unsigned)((totB + 255) / 256)), dim3(256), 0, s, phi, kind, ld, dd.N, dd.D,
                     G2, tilesB, static_cast<uint4*>(phiB16));
  return hipGetLastError();
}

// ------------------------------------------------ two-tile skinny GEMM (bf16 Phi)
// One 16-wide group for both tiles: lane (c, h) supplies rows 16g + 8h .. +7
// of column c of the operand block (two float4 of the blocked-4 layout),
// split into a bfloat16 head and tail; the mean column's eight values come
// from LDS.
constexpr int kMaxStageGroups16 = 256;  // 4096 mean values, 32 KiB

__device__ __forceinline__ void mma16_group(const uint4& a0, const uint4& a1, const float4& b0,
                                            const float4& b1, const double4& m0, const double4& m1,
                                            floatx16 (&acc)[2], double (&accm)[2]) {
  const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
  uint32_t hw[4], lw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t h0 = bf16_rne_bits(bv[2 * q]), h1 = bf16_rne_bits(bv[2 * q + 1]);
    const uint32_t l0 = bf16_rne_bits(bv[2 * q] - __uint_as_float(h0 << 16));
    const uint32_t l1 = bf16_rne_bits(bv[2 * q + 1] - __uint_as_float(h1 << 16));
    hw[q] = h0 | (h1 << 16);
    lw[q] = l0 | (l1 << 16);
  }
  const bf16x8 bh = __builtin_bit_cast(bf16x8, make_uint4(hw[0], hw[1], hw[2], hw[3]));
  const bf16x8 bl = __builtin_bit_cast(bf16x8, make_uint4(lw[0], lw[1], lw[2], lw[3]));
  const bf16x8 av0 = __builtin_bit_cast(bf16x8, a0);
  const bf16x8 av1 = __builtin_bit_cast(bf16x8, a1);
  acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av0, bh, acc[0], 0, 0, 0);
  acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av1, bh, acc[1], 0, 0, 0);
  acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av0, bl, acc[0], 0, 0, 0);
  acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av1, bl, acc[1], 0, 0, 0);
  const double m[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
  const uint32_t w0[4] = {a0.x, a0.y, a0.z, a0.w}, w1[4] = {a1.x, a1.y, a1.z, a1.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    accm[0] = fma((double)bf16_lo_as_float(w0[q]), m[2 * q], accm[0]);
    accm[0] = fma((double)bf16_hi_as_float(w0[q]), m[2 * q + 1], accm[0]);
    accm[1] = fma((double)bf16_lo_as_float(w1[q]), m[2 * q], accm[1]);
    accm[1] = fma((double)bf16_hi_as_float(w1[q]), m[2 * q + 1], accm[1]);
  }
}

// Groups [g0, g1) of the two tiles whose chunks start at pa and pa + tstride;
// wave w takes groups g0 + w + WAVES i.  The mean operand of the range is
// staged in LDS first; the vector loads run through a ring of RING groups.
template <int WAVES, int RING>
__device__ __forceinline__ void gemm16x2(const uint4* __restrict__ pa, int64_t tstride, int64_t g0, int64_t g1,
                                         const float4* __restrict__ B4, const double* __restrict__ bm,
                                         floatx16 (&acc)[2], double (&accm)[2]) {
  __shared__ double4 sm[kMaxStageGroups16 * 4];  // [group][half][2] -> 8 values
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 31, h = lane >> 5;
  const int64_t span = g1 - g0;  // host guarantees span <= kMaxStageGroups16
  for (int64_t e = threadIdx.x; e < span * 4; e += blockDim.x)
    sm[e] = *reinterpret_cast<const double4*>(bm + 16 * g0 + 4 * e);
  __syncthreads();
  const int64_t n = span > wave ? (span - wave + WAVES - 1) / WAVES : 0;
  const int64_t gw = g0 + wave;
  const int smw = 4 * wave + 2 * h;  // sm index of step i: smw + 4 WAVES i (+1)
  const uint4* pw = pa + lane;
#define COFEM_G16_LOAD(slot, g)                                 \
  do {                                                          \
    a0[slot] = pw[(g) * 64];                                    \
    a1[slot] = pw[tstride + (g) * 64];                          \
    b0[slot] = B4[(4 * (g) + 2 * h) * 32 + c];                  \
    b1[slot] = B4[(4 * (g) + 2 * h + 1) * 32 + c];              \
  } while (0)
#define COFEM_G16_MMA(slot, i)                                                                  \
  mma16_group(a0[slot], a1[slot], b0[slot], b1[slot], sm[smw + 4 * WAVES * (i)],              \
              sm[smw + 4 * WAVES * (i) + 1], acc, accm)
  uint4 a0[RING], a1[RING];
  float4 b0[RING], b1[RING];
  if (n < 2 * RING) {
    for (int64_t i = 0; i < n; ++i) {
      const int64_t g = gw + (int64_t)WAVES * i;
      COFEM_G16_LOAD(0, g);
      COFEM_G16_MMA(0, i);
    }
  } else {
#pragma unroll
    for (int r = 0; r < RING; ++r) {
      const int64_t g = gw + (int64_t)WAVES * r;
      COFEM_G16_LOAD(r, g);
      __builtin_amdgcn_sched_barrier(0);
    }
    int64_t i0 = 0;
    for (; i0 + 2 * RING <= n; i0 += RING) {
#pragma unroll
      for (int r = 0; r < RING; ++r) {
        COFEM_G16_MMA(r, i0 + r);
        __builtin_amdgcn_sched_barrier(0);
        const int64_t gn = gw + (int64_t)WAVES * (i0 + r + RING);
        COFEM_G16_LOAD(r, gn);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int r = 0; r < RING; ++r) {
      const int64_t i = i0 + r;
      COFEM_G16_MMA(r, i);
      if (i + RING < n) {
        const int64_t gn = gw + (int64_t)WAVES * (i + RING);
        COFEM_G16_LOAD(r, gn);
      }
    }
#pragma unroll
    for (int r = 0; r < RING; ++r) {
      const int64_t i = i0 + RING + r;
      if (i < n) COFEM_G16_MMA(r, i);
    }
  }
#undef COFEM_G16_LOAD
#undef COFEM_G16_MMA
  accm[0] += __shfl_xor(accm[0], 32, 64);
  accm[1] += __shfl_xor(accm[1], 32, 64);
}

// Sums the waves' two tiles through LDS, one tile at a time.  Thread e gets,
// for tile e / 256, the float4 of tile rows 8k + 4h .. +3 of column c
// (k = (e%256)/64, c = e%32, h = (e%64)/32); threads with e%256 < 32 get the
// mean-column sum of row e%256 of that tile.
template <int WAVES>
__device__ __forceinline__ void wg_reduce_x2(const floatx16 (&acc)[2], const double (&accm)[2], float4* out,
                                             double* outm) {
  __shared__ float red[WAVES][16][64];
  __shared__ double redm[WAVES][2][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tt = threadIdx.x >> 8, ee = threadIdx.x & 255;
  if (lane < 32) {
    redm[wave][0][lane] = accm[0];
    redm[wave][1][lane] = accm[1];
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[t][r];
    __syncthreads();
    if (tt == t) {
      const int k = ee >> 6, l = ee & 63;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int w = 0; w < WAVES; ++w)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += red[w][4 * k + q][l];
      *out = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
  if (ee < 32) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) v += redm[w][tt][ee];
    *outm = v;
  }
}

// blocked-4 float4 index of rows 8k + 4h .. +3 (k = e/64, h = (e%64)/32),
// column e%32, of the 32-row tile starting at row0 (e < 256)
__device__ __forceinline__ int64_t tile_f4_16(int64_t row0, int e) {
  const int k = e >> 6, l = e & 63;
  return ((row0 + 8 * k + 4 * (l >> 5)) >> 2) * 32 + (l & 31);
}

// Cross-workgroup split of the reduction of a two-tile block: thread e holds
// the float4 of tile e/256 (and the mean value when e%256 < 32); the last of
// the `nsplit` workgroups adds the partials in split order.
__device__ __forceinline__ bool split_reduce_x2(int nsplit, int split, int64_t row0, int64_t rows_total,
                                                float* __restrict__ part, double* __restrict__ partm,
                                                uint32_t* counter, float4* v, double* vm) {
  if (nsplit == 1) return true;
  const int tt = threadIdx.x >> 8, ee = threadIdx.x & 255;
  const int64_t r0 = row0 + 32 * tt;
  const int64_t i4 = tile_f4_16(r0, ee);
  {
    float* dst = part + ((int64_t)split * (rows_total / 4) * 32 + i4) * 4;
    store_agent(dst + 0, v->x);
    store_agent(dst + 1, v->y);
    store_agent(dst + 2, v->z);
    store_agent(dst + 3, v->w);
  }
  if (ee < 32) store_agent(&partm[(int64_t)split * rows_total + r0 + ee], *vm);
  if (!last_block_ticket(counter, (uint32_t)nsplit)) return false;
  float t4[4] = {0.f, 0.f, 0.f, 0.f};
  double tm = 0.0;
  for (int sp0 = 0; sp0 < nsplit; sp0 += 4) {
    float x[4][4];
    double xm[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int sp = sp0 + u < nsplit ? sp0 + u : sp0;
      const float* src = part + ((int64_t)sp * (rows_total / 4) * 32 + i4) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) x[u][q] = load_agent(src + q);
      xm[u] = ee < 32 ? load_agent(&partm[(int64_t)sp * rows_total + r0 + ee]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (sp0 + u < nsplit) {
#pragma unroll
        for (int q = 0; q < 4; ++q) t4[q] += x[u][q];
        tm += xm[u];
      }
  }
  *v = make_float4(t4[0], t4[1], t4[2], t4[3]);
  if (ee < 32) *vm = tm;
  if (threadIdx.x == 0) store_agent(counter, 0u);
  return true;
}

constexpr int kG16Waves = 8;

// ------------------------------------------------ inner pass 1: W = Phi~ P
template <int RING>
__device__ __forceinline__ void dense16_pass1_body(
    int64_t pair, int split, const uint4* __restrict__ phiA, int64_t G, int64_t gps, int nsplit, int64_t Np,
    const float* __restrict__ P, const double* __restrict__ pm, float* __restrict__ Wpart,
    double* __restrict__ wmpart, float* __restrict__ W, double* __restrict__ wm,
    uint32_t* __restrict__ cnts, CgScalars* __restrict__ st, int apply_only) {
  if (!apply_only && st->stop) return;
  // tiles 2 pair and 2 pair + 1, reduction split `split` of `nsplit`
  const int64_t g0 = split * gps;
  const int64_t g1 = (g0 + gps < G) ? g0 + gps : G;
  floatx16 acc[2];
  double accm[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.0f;
  gemm16x2<kG16Waves, RING>(phiA + 2 * pair * G * 64, G * 64, g0, g1, reinterpret_cast<const float4*>(P), pm,
                            acc, accm);
  float4 v;
  double vm = 0.0;
  wg_reduce_x2<kG16Waves>(acc, accm, &v, &vm);
  const int64_t row0 = pair * 64;
  if (!split_reduce_x2(nsplit, split, row0, Np, Wpart, wmpart, &cnts[pair * kCounterStride], &v, &vm)) return;
  const int tt = threadIdx.x >> 8, ee = threadIdx.x & 255;
  reinterpret_cast<float4*>(W)[tile_f4_16(row0 + 32 * tt, ee)] = v;
  if (ee < 32) wm[row0 + 32 * tt + ee] = vm;
}

template <int RING>
__global__ __launch_bounds__(64 * kG16Waves) void k_dense16_pass1(
    const uint4* __restrict__ phiA, int64_t G, int64_t gps, int nsplit, int64_t Np,
    const float* __restrict__ P, const double* __restrict__ pm, float* __restrict__ Wpart,
    double* __restrict__ wmpart, float* __restrict__ W, double* __restrict__ wm,
    uint32_t* __restrict__ cnts, CgScalars* __restrict__ st, int apply_only) {
  dense16_pass1_body<RING>(blockIdx.x, blockIdx.y, phiA, G, gps, nsplit, Np, P, pm, Wpart, wmpart, W, wm, cnts,
                           st, apply_only);
}

// ------------------------------------------------ inner pass 2: Q = beta Phi~^T W + alpha P, dots
template <int RING>
__device__ __forceinline__ void dense16_pass2_body(
    int64_t pair, int split, int64_t npairs, const uint4* __restrict__ phiB, int64_t G2, int64_t gps, int nsplit,
    int64_t Dp, const float* __restrict__ W, const double* __restrict__ wm, const float* __restrict__ P,
    const double* __restrict__ pm, const float* __restrict__ R, const double* __restrict__ rm,
    const float* __restrict__ alpha, double beta, float* __restrict__ Qpart, double* __restrict__ qmpart,
    float* __restrict__ Q, double* __restrict__ qm, double* __restrict__ parts, uint32_t* __restrict__ cnts,
    uint32_t* __restrict__ split_cnts, CgScalars* __restrict__ st, int apply_only,
    const float* __restrict__ minv = nullptr) {
  if (!apply_only && st->stop) return;
  const CgCtl ctl = load_cg_ctl(st);
  constexpr int nc = kDenseKP + 1;
  const int64_t g0 = split * gps;
  const int64_t g1 = (g0 + gps < G2) ? g0 + gps : G2;
  floatx16 acc[2];
  double accm[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.0f;
  gemm16x2<kG16Waves, RING>(phiB + 2 * pair * G2 * 64, G2 * 64, g0, g1, reinterpret_cast<const float4*>(W), wm,
                            acc, accm);
  float4 v;
  double vm = 0.0;
  wg_reduce_x2<kG16Waves>(acc, accm, &v, &vm);
  const int64_t d0 = pair * 64;
  if (!split_reduce_x2(nsplit, split, d0, Dp, Qpart, qmpart, &split_cnts[pair * kCounterStride], &v, &vm)) return;

  __shared__ double sdots[3][512];
  __shared__ double smean[3][64];
  __shared__ double mine[3 * nc], tot[3 * nc];
  const int e = threadIdx.x, tt = e >> 8, ee = e & 255;
  const int64_t dt = d0 + 32 * tt;
  {
    const int64_t i4 = tile_f4_16(dt, ee);
    const int64_t dq = dt + 8 * (ee >> 6) + 4 * ((ee & 63) >> 5);  // first of four coordinates
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
      float4 mq = q;  // M^-1 q (del and eta of the preconditioned step)
      if (minv) {
        const float4 mv = *reinterpret_cast<const float4*>(minv + dq);
        mq = make_float4(mv.x * q.x, mv.y * q.y, mv.z * q.z, mv.w * q.w);
      }
      sdots[1][e] = (double)r.x * mq.x + (double)r.y * mq.y + (double)r.z * mq.z + (double)r.w * mq.w;
      sdots[2][e] = (double)q.x * mq.x + (double)q.y * mq.y + (double)q.z * mq.z + (double)q.w * mq.w;
    }
  }
  if (ee < 32) {
    const int64_t d = dt + ee;
    const double p = pm[d];
    const double q = beta * vm + (double)alpha[d] * p;
    const double mq = minv ? (double)minv[d] * q : q;
    qm[d] = q;
    smean[0][32 * tt + ee] = p * q;
    smean[1][32 * tt + ee] = rm[d] * mq;
    smean[2][32 * tt + ee] = q * mq;
  }
  if (apply_only) return;
  __syncthreads();
  if (e < 3 * kDenseKP) {  // column cc: 16 entries, tile-major, then as in the float32 pass
    const int kind = e / kDenseKP, cc = e % kDenseKP;
    double sacc = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < 8; ++q) sacc += sdots[kind][256 * t + 64 * (q >> 1) + 32 * (q & 1) + cc];
    mine[kind * nc + cc] = sacc;
  } else if (e >= 128 && e < 131) {
    const int kind = e - 128;
    double sacc = 0.0;
    for (int i = 0; i < 64; ++i) sacc += smean[kind][i];
    mine[kind * nc + kDenseKP] = sacc;
  }
  __syncthreads();
  if (!tree_reduce(parts, cnts, pair, npairs, 3 * nc, mine, tot)) return;
  finish_step(st, tot, ctl);
}

template <int RING>
__global__ __launch_bounds__(64 * kG16Waves) void k_dense16_pass2(
    const uint4* __restrict__ phiB, int64_t G2, int64_t gps, int nsplit, int64_t Dp,
    const float* __restrict__ W, const double* __restrict__ wm, const float* __restrict__ P,
    const double* __restrict__ pm, const float* __restrict__ R, const double* __restrict__ rm,
    const float* __restrict__ alpha, double beta, float* __restrict__ Qpart, double* __restrict__ qmpart,
    float* __restrict__ Q, double* __restrict__ qm, double* __restrict__ parts, uint32_t* __restrict__ cnts,
    uint32_t* __restrict__ split_cnts, CgScalars* __restrict__ st, int apply_only, const float* __restrict__ minv) {
  dense16_pass2_body<RING>(blockIdx.x, blockIdx.y, gridDim.x, phiB, G2, gps, nsplit, Dp, W, wm, P, pm, R, rm, alpha,
                           beta, Qpart, qmpart, Q, qm, parts, cnts, split_cnts, st, apply_only, minv);
}

// Splits of a low-precision pass: ~256 workgroups of two tiles each (one
// 512-thread workgroup fits a CU at this kernel's register and LDS use),
// within the LDS staging limit of the mean operand.
int dense16_split(int64_t pairs, int64_t groups) {
  int64_t s = (256 + pairs - 1) / pairs;
  const int64_t most = groups / (8 * kG16Waves);
  if (s > most) s = most;
  if (s > 16) s = 16;
  const int64_t least = (groups + kMaxStageGroups16 - 1) / kMaxStageGroups16;
  if (s < least) s = least;
  return (int)(s < 1 ? 1 : s);
}

bool dense16_split_ok(int64_t groups, int splits) {
  return splits >= 1 && (groups + splits - 1) / splits <= kMaxStageGroups16;
}

hipError_t dense16_pass1(const DenseDims& dd, const void* phiA16, const float* P, const double* pm,
                         float* Wpart, double* wmpart, float* W, double* wm, uint32_t* cnts, CgScalars* st,
                         int apply_only, hipStream_t s) {
  const int64_t pairs = dd.Np / 64, G = dd.Dp / 16;
  if (!dense16_split_ok(G, dd.S1h)) return hipErrorInvalidValue;
  const int64_t gps = (G + dd.S1h - 1) / dd.S1h;
  hipLaunchKernelGGL(k_dense16_pass1<4>, dim3((unsigned)pairs, (unsigned)dd.S1h), dim3(64 * kG16Waves), 0, s,
                     static_cast<const uint4*>(phiA16), G, gps, dd.S1h, dd.Np, P, pm, Wpart, wmpart, W, wm,
                     cnts, st, apply_only);
  return hipGetLastError();
}

hipError_t dense16_pass2(const DenseDims& dd, const void* phiB16, const float* W, const double* wm,
                         const float* P, const double* pm, const float* R, const double* rm, const float* alpha,
                         double beta, float* Qpart, double* qmpart, float* Q, double* qm, double* gpart,
                         uint32_t* counter, uint32_t* split_cnts, CgScalars* st, int apply_only, hipStream_t s,
                         const float* minv) {
  const int64_t pairs = dd.Dp / 64, G2 = dd.Np / 16;
  if (!dense16_split_ok(G2, dd.S2h)) return hipErrorInvalidValue;
  const int64_t gps = (G2 + dd.S2h - 1) / dd.S2h;
  hipLaunchKernelGGL(k_dense16_pass2<4>, dim3((unsigned)pairs, (unsigned)dd.S2h), dim3(64 * kG16Waves), 0, s,
                     static_cast<const uint4*>(phiB16), G2, gps, dd.S2h, dd.Dp, W, wm, P, pm, R, rm, alpha, beta,
                     Qpart, qmpart, Q, qm, gpart, counter, split_cnts, st, apply_only, minv);
  return hipGetLastError();
}

// ------------------------------------------------ iterative refinement glue
// Warm start of a refinement: the probe columns of Xt become
// max(s_prev, 0) (.) p_k for the probes of EM iteration t (x_k ~ Sigma p_k from
// the previous diagonal estimate); the float64 mean column keeps the previous
// E-step's mean, which Xt still holds.
__global__ __launch_bounds__(256) void k_dense_warm_start(int64_t D, int64_t Dp, uint64_t seed, int t, int K,
                                                          const float* __restrict__ sprev, float* __restrict__ Xt) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    const int c = (int)(e4 & 31);
    const int64_t d0 = (e4 >> 5) * 4;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t d = d0 + i;
      v[i] = (d < D && c < K) ? fmaxf(sprev[d], 0.0f) * probe_sign(seed, (uint32_t)t, (uint32_t)c, (uint64_t)d)
                              : 0.0f;
    }
    reinterpret_cast<float4*>(Xt)[e4] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

hipError_t dense_warm_start(const DenseDims& dd, uint64_t seed, int t, int K, const float* sprev, float* Xt,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_dense_warm_start, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.D, dd.Dp, seed, t, K,
                     sprev, Xt);
  return hipGetLastError();
}

// Xt += Xi over the blocked-4 probe block and the float64 mean column.
__global__ __launch_bounds__(256) void k_dense_ir_accumulate(int64_t Dp, float* __restrict__ Xt,
                                                             const float* __restrict__ Xi,
                                                             double* __restrict__ xtm,
                                                             const double* __restrict__ xim) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    float4 a = reinterpret_cast<float4*>(Xt)[e4];
    const float4 b = reinterpret_cast<const float4*>(Xi)[e4];
    a.x += b.x;
    a.y += b.y;
    a.z += b.z;
    a.w += b.w;
    reinterpret_cast<float4*>(Xt)[e4] = a;
  }
  for (int64_t d = gtid; d < Dp; d += gstride) xtm[d] += xim[d];
}

hipError_t dense_ir_accumulate(const DenseDims& dd, float* Xt, const float* Xi, double* xtm, const double* xim,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_dense_ir_accumulate, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.Dp, Xt, Xi, xtm,
                     xim);
  return hipGetLastError();
}

// Outer residual of the refinement: with Q = A Xt (float32 Phi passes) and B
// regenerated (probes of EM iteration t in rows d < D, b0 for the mean),
// R = B - Q, P = R, Xi = 0; rho_c = ||r_c||^2 (float64 sums of the stored
// values).  With a Jacobi diagonal minv: P = M^-1 R and the sums r^T z and
// r^T r (finish_ir_residual_pcg).  The finish sets up the next inner solve: reference norm ||R||_F,
// iteration count 0, cap `limit`, and the true ratio ||R||_F / ||B||_F.
__global__ __launch_bounds__(256) void k_dense_ir_residual(
    int64_t D, int64_t Dp, uint64_t seed, int t, int K, const double* __restrict__ b0, const float* __restrict__ Q,
    const double* __restrict__ qm, float* __restrict__ Xi, float* __restrict__ R, float* __restrict__ P,
    double* __restrict__ xim, double* __restrict__ rm, double* __restrict__ pm, double* __restrict__ parts,
    uint32_t* cnts, CgScalars* st, int limit, const float* __restrict__ minv) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  const int c = threadIdx.x & 31;
  double acc = 0.0, accz = 0.0;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    const float4 q = reinterpret_cast<const float4*>(Q)[e4];
    const int64_t d0 = (e4 >> 5) * 4;
    const float qv[4] = {q.x, q.y, q.z, q.w};
    const float4 mv = minv ? *reinterpret_cast<const float4*>(minv + d0) : make_float4(1.f, 1.f, 1.f, 1.f);
    const float m4[4] = {mv.x, mv.y, mv.z, mv.w};
    float rv[4], zv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t d = d0 + i;
      const float b = (c < K && d < D) ? probe_sign(seed, (uint32_t)t, (uint32_t)c, (uint64_t)d) : 0.0f;
      rv[i] = b - qv[i];
      zv[i] = m4[i] * rv[i];
      acc += (double)rv[i] * (double)rv[i];
      accz += (double)rv[i] * (double)zv[i];
    }
    reinterpret_cast<float4*>(R)[e4] = make_float4(rv[0], rv[1], rv[2], rv[3]);
    reinterpret_cast<float4*>(P)[e4] = make_float4(zv[0], zv[1], zv[2], zv[3]);
    reinterpret_cast<float4*>(Xi)[e4] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  double accm = 0.0, accmz = 0.0;
  for (int64_t d = gtid; d < Dp; d += gstride) {
    const double r = b0[d] - qm[d];
    const double z = minv ? (double)minv[d] * r : r;
    rm[d] = r;
    pm[d] = z;
    xim[d] = 0.0;
    accm += r * r;
    accmz += r * z;
  }
  constexpr int nc = kDenseKP + 1;
  __shared__ double mine[2 * nc], tot[2 * nc];
  if (!minv) {
    dense_block_sums(acc, accm, mine);
    if (!tree_reduce(parts, cnts, blockIdx.x, gridDim.x, nc, mine, tot)) return;
    finish_ir_residual(st, tot, limit);
    return;
  }
  dense_block_sums(accz, accmz, mine);
  dense_block_sums(acc, accm, mine + nc);
  if (!tree_reduce(parts, cnts, blockIdx.x, gridDim.x, 2 * nc, mine, tot)) return;
  finish_ir_residual_pcg(st, tot, limit);
}

hipError_t dense_ir_residual(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0, const float* Q,
                             const double* qm, float* Xi, float* R, float* P, double* xim, double* rm, double* pm,
                             double* parts, uint32_t* cnts, CgScalars* st, int limit, hipStream_t s,
                             const float* minv) {
  hipLaunchKernelGGL(k_dense_ir_residual, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.D, dd.Dp, seed, t, K,
                     b0, Q, qm, Xi, R, P, xim, rm, pm, parts, cnts, st, limit, minv);
  return hipGetLastError();
}

}  // namespace cofem

namespace cofem {

// ------------------------------------------------ batched form: grouped passes
// One launch covers every problem's (tile pair, split) work items; a block
// reads its item and its problem's descriptor and runs the single-problem
// pass body on them (the problem's own stop flag, counters and tree).
__global__ __launch_bounds__(64 * kG16Waves) void k_batch_pass1(const BatchItem* __restrict__ items,
                                                                const BatchProblem* __restrict__ probs,
                                                                int apply_only) {
  const BatchItem it = items[blockIdx.x];
  const BatchProblem& p = probs[it.prob];
  const int64_t G = p.Dp / 16;
  const int64_t gps = (G + p.S1 - 1) / p.S1;
  dense16_pass1_body<4>(it.a, it.b, static_cast<const uint4*>(p.phiA16), G, gps, p.S1, p.Np, p.P, p.pm, p.Wpart,
                        p.wmpart, p.W, p.wm, p.cnt_split1, p.st, apply_only);
}

__global__ __launch_bounds__(64 * kG16Waves) void k_batch_pass2(const BatchItem* __restrict__ items,
                                                                const BatchProblem* __restrict__ probs, double beta,
                                                                int apply_only) {
  const BatchItem it = items[blockIdx.x];
  const BatchProblem& p = probs[it.prob];
  const int64_t G2 = p.Np / 16;
  const int64_t gps = (G2 + p.S2 - 1) / p.S2;
  dense16_pass2_body<4>(it.a, it.b, p.npairs2, static_cast<const uint4*>(p.phiB16), G2, gps, p.S2, p.Dp, p.W, p.wm,
                        p.P, p.pm, p.R, p.rm, p.alpha, beta, p.Qpart, p.qmpart, p.Q, p.qm, p.parts_pass, p.cnts_pass,
                        p.cnt_split2, p.st, apply_only);
}

hipError_t batch_pass1(const BatchItem* items, int n, const BatchProblem* probs, int apply_only, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_pass1, dim3((unsigned)n), dim3(64 * kG16Waves), 0, s, items, probs, apply_only);
  return hipGetLastError();
}

hipError_t batch_pass2(const BatchItem* items, int n, const BatchProblem* probs, double beta, int apply_only,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_pass2, dim3((unsigned)n), dim3(64 * kG16Waves), 0, s, items, probs, beta, apply_only);
  return hipGetLastError();
}

}  // namespace cofem
