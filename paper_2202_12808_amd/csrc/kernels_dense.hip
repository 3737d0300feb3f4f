// Dense-dictionary kernels of the CoFEM E-step (Sec. 3.1-3.2 of arXiv 2202.12808).
//
// Per CG iteration the operator A P = beta Phi^T (Phi P) + alpha (.) P is applied
// to all K+1 columns at once (mat-vecs replaced by mat-mats, Sec. 3.2) as two
// skinny GEMMs on the matrix cores with v_mfma_f32_16x16x4f32:
//   pass 1  W = Phi P          one workgroup per 16-row tile of Phi,
//   pass 2  Q = Phi^T W + ...  one workgroup per 16-coordinate tile,
// each workgroup splitting the reduction over its waves and summing the
// waves' tiles in LDS.  The 32 probe slots are two 16-column MFMA blocks.
// The mean column (column K of Eq. 7) rides along on the vector ALU in
// float64 -- one FMA per Phi element already in registers -- so it costs no
// extra Phi traffic.  Both passes stream Phi from HBM once; every wave keeps a
// four-deep ring of outstanding loads (Phi fragment, B fragment, mean values)
// so that enough bytes are in flight to cover the memory latency.
//
// Layouts (all owned by the library):
//  * phiA: for 16-row tile t and 16-column group g, one contiguous 1 KiB chunk;
//    lane l holds Phi[16 t + l%16][16 g + 4 (l/16) + s], s = 0..3, i.e. the A
//    operand of four consecutive MFMAs (k index l/16 of MFMA s <-> column
//    16g + 4(l/16) + s).
//  * phiB: the same for Phi^T: lane l holds Phi[16 g + 4 (l/16) + s][16 t + l%16].
//  * probe-column state X, R, P, Q and W: blocked-4 (see DenseDims), whose
//    float4 at ((k/4) * 32 + c) is exactly the B fragment of lane (c%16, k%16/4)
//    and whose C-result rows 4(l/16)..+3 of column c form one float4.
//  * mean-column state: float64 vectors.
#include "cofem_internal.h"

namespace cofem {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kRing = 4;  // outstanding groups per wave

// --------------------------------------------------------------- packing
__global__ void k_pack_a16(const float* __restrict__ phi, int64_t ld, int64_t N, int64_t D,
                           int64_t G, int64_t tiles, float4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tiles * G * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int64_t g = rest % G, t = rest / G;
  const int64_t n = 16 * t + (lane & 15);
  const int64_t d0 = 16 * g + 4 * (lane >> 4);
  float v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = (n < N && d0 + s < D) ? phi[n * ld + d0 + s] : 0.0f;
  out[idx] = make_float4(v[0], v[1], v[2], v[3]);
}

__global__ void k_pack_b16(const float* __restrict__ phi, int64_t ld, int64_t N, int64_t D,
                           int64_t G2, int64_t tiles, float4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tiles * G2 * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int64_t g = rest % G2, t = rest / G2;
  const int64_t d = 16 * t + (lane & 15);
  const int64_t n0 = 16 * g + 4 * (lane >> 4);
  float v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = (n0 + s < N && d < D) ? phi[(n0 + s) * ld + d] : 0.0f;
  out[idx] = make_float4(v[0], v[1], v[2], v[3]);
}

hipError_t dense_pack(const float* phi, int64_t ld, const DenseDims& dd, float* phiA, float* phiB,
                      hipStream_t s) {
  const int64_t G = dd.Dp / 16, tilesA = dd.Np / 16;
  const int64_t totA = tilesA * G * 64;
  hipLaunchKernelGGL(k_pack_a16, dim3((unsigned)((totA + 255) / 256)), dim3(256), 0, s, phi, ld, dd.N,
                     dd.D, G, tilesA, reinterpret_cast<float4*>(phiA));
  const int64_t G2 = dd.Np / 16, tilesB = dd.Dp / 16;
  const int64_t totB = tilesB * G2 * 64;
  hipLaunchKernelGGL(k_pack_b16, dim3((unsigned)((totB + 255) / 256)), dim3(256), 0, s, phi, ld, dd.N,
                     dd.D, G2, tilesB, reinterpret_cast<float4*>(phiB));
  return hipGetLastError();
}

// ------------------------------------------------- b0 = beta Phi^T y (Eq. 5)
__global__ void k_dense_b0(const float* __restrict__ phi, int64_t ld, const float* __restrict__ y,
                           double beta, int64_t N, int64_t D, int64_t Dp, double* __restrict__ b0) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= Dp) return;
  double acc = 0.0;
  if (d < D)
    for (int64_t n = 0; n < N; ++n) acc = fma((double)phi[n * ld + d], (double)y[n], acc);
  b0[d] = beta * acc;
}

hipError_t dense_b0(const float* phi, int64_t ld, const float* y, double beta, const DenseDims& dd,
                    double* b0, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_b0, dim3((unsigned)((dd.Dp + 255) / 256)), dim3(256), 0, s, phi, ld, y,
                     beta, dd.N, dd.D, dd.Dp, b0);
  return hipGetLastError();
}

// ------------------------------------------------ per-block column sums
// Thread tid owns probe column tid & 31 (acc) and a share of the mean column
// (accm); leaves the block's 33 sums in out_sh (256-thread blocks).
__device__ __forceinline__ void dense_block_sums(double acc, double accm, double* out_sh) {
  __shared__ double sh[kThreads];
  __shared__ double shm[8];
  sh[threadIdx.x] = acc;
  const double m = block_sum(accm, shm);  // synchronises
  if (threadIdx.x < kDenseKP) {
    double v = 0.0;
    for (int t = threadIdx.x; t < kThreads; t += kDenseKP) v += sh[t];
    out_sh[threadIdx.x] = v;
  } else if (threadIdx.x == kDenseKP) {
    out_sh[kDenseKP] = m;
  }
  __syncthreads();
}

int dense_update_blocks(const DenseDims& dd) {
  const int64_t want = (dd.Dp * 8 + 4 * 256 - 1) / (4 * 256);
  return (int)(want < 1 ? 1 : (want > 256 ? 256 : want));
}

// ------------------------------------------------ initial residual R = P = B (Eq. 7)
__global__ __launch_bounds__(256) void k_dense_init(int64_t D, int64_t Dp, uint64_t seed, int t,
                                                    int K, const double* __restrict__ b0,
                                                    float* __restrict__ X, float* __restrict__ R,
                                                    float* __restrict__ P, double* __restrict__ xm,
                                                    double* __restrict__ rm,
                                                    double* __restrict__ pm,
                                                    double* __restrict__ parts, uint32_t* cnts,
                                                    CgScalars* st) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  const int c = threadIdx.x & 31;
  double acc = 0.0;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    const int64_t d0 = (e4 >> 5) * 4;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = (d0 + i < D && c < K) ? probe_sign(seed, (uint32_t)t, (uint32_t)c, (uint64_t)(d0 + i)) : 0.0f;
      acc += (double)v[i] * (double)v[i];
    }
    const float4 r = make_float4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<float4*>(R)[e4] = r;
    reinterpret_cast<float4*>(P)[e4] = r;
    reinterpret_cast<float4*>(X)[e4] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  double accm = 0.0;
  for (int64_t d = gtid; d < Dp; d += gstride) {
    const double b = b0[d];
    rm[d] = b;
    pm[d] = b;
    xm[d] = 0.0;
    accm += b * b;
  }
  __shared__ double mine[kDenseKP + 1], tot[kDenseKP + 1];
  dense_block_sums(acc, accm, mine);
  if (!tree_reduce(parts, cnts, blockIdx.x, gridDim.x, kDenseKP + 1, mine, tot)) return;
  finish_init(st, tot);
}

hipError_t dense_init(const DenseDims& dd, uint64_t seed, int t, int K, const double* b0,
                      float* X, float* R, float* P, double* xm, double* rm, double* pm,
                      double* parts, uint32_t* cnts, CgScalars* st, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_init, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.D, dd.Dp, seed,
                     t, K, b0, X, R, P, xm, rm, pm, parts, cnts, st);
  return hipGetLastError();
}

// ------------------------------------------------ skinny GEMM tile (16 x 32 + mean)
// The workgroup's WAVES waves split the groups [0, G) of its tile; returns the
// workgroup-summed tile in red_out (thread e < 128: rows 4(l/16)..+3 of
// column 16(e/64) + l%16, l = e%64, as a float4) and, for e < 16, the
// mean-column sum of tile row e.
template <int WAVES>
__device__ __forceinline__ void gemm16(const float4* __restrict__ pa, int64_t G,
                                       const float4* __restrict__ B4, const double* __restrict__ bm,
                                       float4* red_out, double* redm_out) {
  __shared__ floatx4 red[WAVES][2][64];
  __shared__ double redm[WAVES][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kk = lane >> 4;
  const int64_t per = (G + WAVES - 1) / WAVES;
  const int64_t g0 = wave * per;
  const int64_t g1 = (g0 + per < G) ? g0 + per : G;

  floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  double accm = 0.0;
  float4 a[kRing], b0r[kRing], b1r[kRing];
  double2 m0r[kRing], m1r[kRing];
  const float4* paw = pa + lane;
#pragma unroll
  for (int i = 0; i < kRing; ++i) {
    const int64_t g = g0 + i;
    if (g < g1) {
      a[i] = paw[g * 64];
      b0r[i] = B4[(4 * g + kk) * 32 + j];
      b1r[i] = B4[(4 * g + kk) * 32 + 16 + j];
      m0r[i] = *reinterpret_cast<const double2*>(bm + 16 * g + 4 * kk);
      m1r[i] = *reinterpret_cast<const double2*>(bm + 16 * g + 4 * kk + 2);
    }
  }
  for (int64_t g = g0; g < g1; g += kRing) {
#pragma unroll
    for (int i = 0; i < kRing; ++i) {
      const int64_t gi = g + i;
      if (gi < g1) {
        const float4 av = a[i], b0 = b0r[i], b1 = b1r[i];
        const double2 m0 = m0r[i], m1 = m1r[i];
        const int64_t gn = gi + kRing;
        if (gn < g1) {
          a[i] = paw[gn * 64];
          b0r[i] = B4[(4 * gn + kk) * 32 + j];
          b1r[i] = B4[(4 * gn + kk) * 32 + 16 + j];
          m0r[i] = *reinterpret_cast<const double2*>(bm + 16 * gn + 4 * kk);
          m1r[i] = *reinterpret_cast<const double2*>(bm + 16 * gn + 4 * kk + 2);
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, b0.x, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, b1.x, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, b0.y, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, b1.y, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, b0.z, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, b1.z, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, b0.w, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, b1.w, acc1, 0, 0, 0);
        accm = fma((double)av.x, m0.x, accm);
        accm = fma((double)av.y, m0.y, accm);
        accm = fma((double)av.z, m1.x, accm);
        accm = fma((double)av.w, m1.y, accm);
      }
    }
  }
  // mean column: the four k-quarters of tile row j
  accm += __shfl_xor(accm, 16, 64);
  accm += __shfl_xor(accm, 32, 64);
  red[wave][0][lane] = acc0;
  red[wave][1][lane] = acc1;
  if (kk == 0) redm[wave][j] = accm;
  __syncthreads();
  if (threadIdx.x < 128) {
    const int cb = threadIdx.x >> 6, l = threadIdx.x & 63;
    floatx4 v = red[0][cb][l];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) v += red[w][cb][l];
    *red_out = make_float4(v[0], v[1], v[2], v[3]);
  }
  if (threadIdx.x < 16) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) v += redm[w][threadIdx.x];
    *redm_out = v;
  }
}

// ------------------------------------------------ pass 1: W = Phi P
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_dense_pass1(const float4* __restrict__ phiA,
                                                            int64_t G, const float* __restrict__ P,
                                                            const double* __restrict__ pm,
                                                            float* __restrict__ W,
                                                            double* __restrict__ wm,
                                                            CgScalars* __restrict__ st,
                                                            int apply_only) {
  if (!apply_only && st->stop) return;
  const int64_t tile = blockIdx.x;
  float4 v;
  double vm;
  gemm16<WAVES>(phiA + tile * G * 64, G, reinterpret_cast<const float4*>(P), pm, &v, &vm);
  const int64_t n0 = tile * 16;
  if (threadIdx.x < 128) {
    const int cb = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int col = 16 * cb + (l & 15);
    reinterpret_cast<float4*>(W)[((n0 >> 2) + (l >> 4)) * 32 + col] = v;
  }
  if (threadIdx.x < 16) wm[n0 + threadIdx.x] = vm;
}

hipError_t dense_pass1(const DenseDims& dd, const float* phiA, const float* P, const double* pm,
                       float* W, double* wm, CgScalars* st, int apply_only, hipStream_t s) {
  const int64_t tiles = dd.Np / 16, G = dd.Dp / 16;
  const float4* pa = reinterpret_cast<const float4*>(phiA);
#define COFEM_PASS1(WV)                                                                             \
  hipLaunchKernelGGL(k_dense_pass1<WV>, dim3((unsigned)tiles), dim3(64 * WV), 0, s, pa, G, P, pm, W, wm, \
                     st, apply_only)
  switch (dd.waves1) {
    case 4: COFEM_PASS1(4); break;
    case 8: COFEM_PASS1(8); break;
    default: COFEM_PASS1(16); break;
  }
#undef COFEM_PASS1
  return hipGetLastError();
}

// ------------------------------------------------ pass 2: Q = beta Phi^T W + alpha (.) P
// The epilogue also forms the per-column dots gam = p^T q, del = r^T q and
// eta = q^T q; the tree reduction's final workgroup turns them into a_c, b_c.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_dense_pass2(
    const float4* __restrict__ phiB, int64_t G2, const float* __restrict__ W,
    const double* __restrict__ wm, const float* __restrict__ P, const double* __restrict__ pm,
    const float* __restrict__ R, const double* __restrict__ rm, const float* __restrict__ alpha,
    double beta, float* __restrict__ Q, double* __restrict__ qm, double* __restrict__ parts,
    uint32_t* __restrict__ cnts, CgScalars* __restrict__ st, int apply_only) {
  if (!apply_only && st->stop) return;
  constexpr int nc = kDenseKP + 1;
  const int64_t tile = blockIdx.x;
  float4 v;
  double vm;
  gemm16<WAVES>(phiB + tile * G2 * 64, G2, reinterpret_cast<const float4*>(W), wm, &v, &vm);
  const int64_t d0 = tile * 16;
  __shared__ double mine[3 * nc], tot[3 * nc];
  if (threadIdx.x < 128) {
    const int cb = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int col = 16 * cb + (l & 15);
    const int64_t dq = d0 + 4 * (l >> 4);  // first of four coordinates
    const int64_t i4 = (dq >> 2) * 32 + col;
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
      double g = (double)p.x * q.x + (double)p.y * q.y + (double)p.z * q.z + (double)p.w * q.w;
      double dl = (double)r.x * q.x + (double)r.y * q.y + (double)r.z * q.z + (double)r.w * q.w;
      double et = (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z + (double)q.w * q.w;
      // sum over the four row groups of this column (lanes l, l^16, l^32, l^48)
      g += __shfl_xor(g, 16, 64);
      g += __shfl_xor(g, 32, 64);
      dl += __shfl_xor(dl, 16, 64);
      dl += __shfl_xor(dl, 32, 64);
      et += __shfl_xor(et, 16, 64);
      et += __shfl_xor(et, 32, 64);
      if ((l >> 4) == 0) {
        mine[col] = g;
        mine[nc + col] = dl;
        mine[2 * nc + col] = et;
      }
    }
  }
  if (threadIdx.x < 64) {  // mean column, lanes 0..15 of wave 0
    double g = 0.0, dl = 0.0, et = 0.0;
    if (threadIdx.x < 16) {
      const int64_t d = d0 + threadIdx.x;
      const double p = pm[d];
      const double q = beta * vm + (double)alpha[d] * p;
      qm[d] = q;
      g = p * q;
      dl = rm[d] * q;
      et = q * q;
    }
    if (!apply_only) {
      for (int off = 8; off > 0; off >>= 1) {
        g += __shfl_xor(g, off, 64);
        dl += __shfl_xor(dl, off, 64);
        et += __shfl_xor(et, off, 64);
      }
      if (threadIdx.x == 0) {
        mine[kDenseKP] = g;
        mine[nc + kDenseKP] = dl;
        mine[2 * nc + kDenseKP] = et;
      }
    }
  }
  if (apply_only) return;
  __syncthreads();
  if (!tree_reduce(parts, cnts, tile, gridDim.x, 3 * nc, mine, tot)) return;
  finish_step(st, tot);
}

hipError_t dense_pass2(const DenseDims& dd, const float* phiB, const float* W, const double* wm,
                       const float* P, const double* pm, const float* R, const double* rm,
                       const float* alpha, double beta, float* Q, double* qm, double* gpart,
                       uint32_t* counter, CgScalars* st, int apply_only, hipStream_t s) {
  const int64_t tiles = dd.Dp / 16, G2 = dd.Np / 16;
  const float4* pb = reinterpret_cast<const float4*>(phiB);
#define COFEM_PASS2(WV)                                                                               \
  hipLaunchKernelGGL(k_dense_pass2<WV>, dim3((unsigned)tiles), dim3(64 * WV), 0, s, pb, G2, W, wm, P, pm, \
                     R, rm, alpha, beta, Q, qm, gpart, counter, st, apply_only)
  switch (dd.waves2) {
    case 4: COFEM_PASS2(4); break;
    case 8: COFEM_PASS2(8); break;
    default: COFEM_PASS2(16); break;
  }
#undef COFEM_PASS2
  return hipGetLastError();
}

int dense_pass_waves(int64_t tiles) {
  if (tiles >= 1024) return 4;
  if (tiles >= 512) return 8;
  return 16;
}

// ------------------------------------------------ CG update
// x += a p ; r -= a q ; p <- r + b p ; rho' = ||r||^2 and the stop test.
__global__ __launch_bounds__(256) void k_dense_update(int64_t Dp, float* __restrict__ X,
                                                      float* __restrict__ R, float* __restrict__ P,
                                                      const float* __restrict__ Q,
                                                      double* __restrict__ xm,
                                                      double* __restrict__ rm,
                                                      double* __restrict__ pm,
                                                      const double* __restrict__ qm,
                                                      double* __restrict__ parts, uint32_t* cnts,
                                                      CgScalars* st) {
  if (st->stop) return;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  const int c = threadIdx.x & 31;
  const float a = (float)st->a[c], b = (float)st->b[c];
  const double am = st->a[kDenseKP], bmm = st->b[kDenseKP];
  double acc = 0.0;
  for (int64_t e4 = gtid; e4 < Dp * 8; e4 += gstride) {
    float4 x = reinterpret_cast<float4*>(X)[e4];
    float4 r = reinterpret_cast<float4*>(R)[e4];
    float4 p = reinterpret_cast<float4*>(P)[e4];
    const float4 q = reinterpret_cast<const float4*>(Q)[e4];
    x.x = fmaf(a, p.x, x.x);
    x.y = fmaf(a, p.y, x.y);
    x.z = fmaf(a, p.z, x.z);
    x.w = fmaf(a, p.w, x.w);
    r.x = fmaf(-a, q.x, r.x);
    r.y = fmaf(-a, q.y, r.y);
    r.z = fmaf(-a, q.z, r.z);
    r.w = fmaf(-a, q.w, r.w);
    p.x = fmaf(b, p.x, r.x);
    p.y = fmaf(b, p.y, r.y);
    p.z = fmaf(b, p.z, r.z);
    p.w = fmaf(b, p.w, r.w);
    reinterpret_cast<float4*>(X)[e4] = x;
    reinterpret_cast<float4*>(R)[e4] = r;
    reinterpret_cast<float4*>(P)[e4] = p;
    acc += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
  }
  double accm = 0.0;
  for (int64_t d = gtid; d < Dp; d += gstride) {
    const double p = pm[d];
    xm[d] = fma(am, p, xm[d]);
    const double r = fma(-am, qm[d], rm[d]);
    rm[d] = r;
    pm[d] = fma(bmm, p, r);
    accm += r * r;
  }
  __shared__ double mine[kDenseKP + 1], tot[kDenseKP + 1];
  dense_block_sums(acc, accm, mine);
  if (!tree_reduce(parts, cnts, blockIdx.x, gridDim.x, kDenseKP + 1, mine, tot)) return;
  finish_update(st, tot);
}

hipError_t dense_update(const DenseDims& dd, float* X, float* R, float* P, const float* Q,
                        double* xm, double* rm, double* pm, const double* qm, double* parts,
                        uint32_t* cnts, CgScalars* st, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_update, dim3(dense_update_blocks(dd)), dim3(256), 0, s, dd.Dp, X, R, P,
                     Q, xm, rm, pm, qm, parts, cnts, st);
  return hipGetLastError();
}

// ------------------------------------------------ diagonal estimate + M-step (Eq. 6, Eq. 8)
__global__ __launch_bounds__(256) void k_dense_mstep(int64_t D, uint64_t seed, int t, int K,
                                                     const float* __restrict__ X,
                                                     const double* __restrict__ xm,
                                                     float* __restrict__ alpha, double alpha_max,
                                                     float* __restrict__ mu,
                                                     float* __restrict__ sdiag, CgScalars* st) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  const double floor_v = 1.0 / alpha_max;
  double clamped = 0.0;
  for (int64_t d = gtid; d < D; d += gstride) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k)
      acc += (double)probe_sign(seed, (uint32_t)t, (uint32_t)k, (uint64_t)d) * (double)X[blk4(d, k)];
    const double s = acc / (double)K;
    const double m = xm[d];
    const double den = m * m + s;
    if (!(den >= floor_v)) clamped += 1.0;
    alpha[d] = (float)(1.0 / (den >= floor_v ? den : floor_v));
    mu[d] = (float)m;
    sdiag[d] = (float)s;
  }
  __shared__ double shm[8];
  const double tot = block_sum(clamped, shm);
  if (threadIdx.x == 0 && tot > 0.0) atomicAdd(&st->n_clamped, (int)tot);
}

hipError_t dense_mstep(const DenseDims& dd, uint64_t seed, int t, int K, const float* X,
                       const double* xm, float* alpha, double alpha_max, float* mu, float* sdiag,
                       CgScalars* st, hipStream_t s) {
  const int64_t want = (dd.D + 255) / 256;
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 2048 ? 2048 : want));
  hipLaunchKernelGGL(k_dense_mstep, dim3(blocks), dim3(256), 0, s, dd.D, seed, t, K, X, xm, alpha,
                     alpha_max, mu, sdiag, st);
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
