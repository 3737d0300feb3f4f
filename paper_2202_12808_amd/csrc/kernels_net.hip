// Learned warm start for convolution dictionaries (the learned form; not in
// the paper).  A small fully convolutional network on the image grid, trained
// on the GPU by the kernels below.  Before EM iteration t it reads the state:
// alpha_t, the previous mean and the previous diagonal estimate.  It predicts
// a start for that E-step's CG solve (run with the Jacobi preconditioner); the
// solve's unchanged stop rule (Sec. 3.2) then corrects and judges the
// prediction.
//
// Definitions (features, network, prediction, loss):
//   d = beta ||h||^2 + alpha (the diagonal of A); features
//     f0 = alpha / d, f1 = mu_prev / rms(mu_prev),
//     f2 = log(clip(s_prev d, 1e-3, 1e3)) / 3, f3 = log(d / (beta ||h||^2)) / 10,
//     f4 = clip(log(d_prev / d), -10, 10) / 10 (d_prev from the previous E-step's alpha);
//   four 3x3 convolutions with circular padding, 5 -> 32 -> 32 -> 32 -> 2
//   channels, ReLU after the first three,
//     out[co][u][v] = b[co] + sum w[co][ci][ky][kx] x[ci][(u+ky-1) mod H][(v+kx-1) mod W];
//   with sb = clip(s_prev d, 0.05, 20):
//   mu_hat = mu_prev (1 + tanh o0), d_hat = exp(clip(o1, -10, 10)) sb / d;
//   with tgt = log(clip(s_t d, 0.05, 20) / sb), each term relative to the
//   untrained network's (the previous iterate's) and f = 1e-4:
//   loss = sum (mu_hat - mu_t)^2 / (sum (mu_prev - mu_t)^2 + f sum mu_t^2)
//          + 0.1 sum (o1 - tgt)^2 / (sum tgt^2 + f HW).
// The untrained network (zero last layer) reproduces the previous iterate,
// so training learns corrections to the non-learned warm start.
// Activations are channel-major float32 images; sums of the loss and of the
// weight gradients are deterministic (fixed-order partials).
#include "cofem.h"
#include "cofem_internal.h"

#include <math.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

namespace cofem {

constexpr int kNetLayers = 4;
constexpr int kNetCh[kNetLayers + 1] = {5, 32, 32, 32, 2};
constexpr int kNetMaxC = 32;
constexpr double kNetLambdaD = 0.1;
constexpr double kNetNormFloor = 1e-4;  // changes below 1% of the mean count as converged
constexpr int kNT = 16;               // pixel tile side
constexpr int kNHalo = kNT + 2;       // tile plus a one-pixel halo
constexpr int kNetWgBlocks = 256;     // blocks of the weight-gradient kernel

__host__ __device__ constexpr int64_t net_layer_params(int l) {
  return (int64_t)kNetCh[l + 1] * kNetCh[l] * 9 + kNetCh[l + 1];
}

__device__ __forceinline__ int nwrap(int x, int n) {
  x %= n;
  return x < 0 ? x + n : x;
}

// ------------------------------------------------ 3x3 circular convolution
// out[co] = b[co] + sum_ci,ky,kx w[co][ci][ky][kx] in[ci][u+ky-1][v+kx-1]
// for COT output channels per block (blockIdx.z selects the group); optional
// ReLU, optional mask (out *= mask > 0: the ReLU derivative of the layer
// below in the backward pass).  One thread per pixel of a 16x16 tile.
template <int COT>
__global__ __launch_bounds__(256) void k_net_conv3(const float* __restrict__ in, int cin, const float* __restrict__ w,
                                                   const float* __restrict__ b, float* __restrict__ out, int cout,
                                                   int H, int W, int relu, const float* __restrict__ mask) {
  __shared__ float s_in[kNetMaxC * kNHalo * kNHalo];
  __shared__ float s_w[COT * kNetMaxC * 9];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int v0 = blockIdx.x * kNT, u0 = blockIdx.y * kNT;
  const int co0 = blockIdx.z * COT;
  const int64_t HW = (int64_t)H * W;
  for (int e = threadIdx.x; e < cin * kNHalo * kNHalo; e += blockDim.x) {
    const int ci = e / (kNHalo * kNHalo), r = e - ci * (kNHalo * kNHalo);
    const int i = r / kNHalo, j = r - i * kNHalo;
    s_in[e] = in[(int64_t)ci * HW + (int64_t)nwrap(u0 + i - 1, H) * W + nwrap(v0 + j - 1, W)];
  }
  for (int e = threadIdx.x; e < COT * cin * 9; e += blockDim.x) {
    const int co = e / (cin * 9);
    s_w[e] = (co0 + co < cout) ? w[(int64_t)(co0 + co) * cin * 9 + (e - co * cin * 9)] : 0.0f;
  }
  __syncthreads();
  const int u = u0 + ty, v = v0 + tx;
  if (u >= H || v >= W) return;
  float acc[COT];
#pragma unroll
  for (int c = 0; c < COT; ++c) acc[c] = (b && co0 + c < cout) ? b[co0 + c] : 0.0f;
  for (int ci = 0; ci < cin; ++ci) {
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const float x = s_in[ci * kNHalo * kNHalo + (ty + ky) * kNHalo + (tx + kx)];
#pragma unroll
        for (int c = 0; c < COT; ++c) acc[c] = fmaf(s_w[(c * cin + ci) * 9 + ky * 3 + kx], x, acc[c]);
      }
  }
  const int64_t p = (int64_t)u * W + v;
#pragma unroll
  for (int c = 0; c < COT; ++c) {
    if (co0 + c >= cout) break;
    float o = acc[c];
    if (relu) o = fmaxf(o, 0.0f);
    if (mask && !(mask[(int64_t)(co0 + c) * HW + p] > 0.0f)) o = 0.0f;
    out[(int64_t)(co0 + c) * HW + p] = o;
  }
}

static hipError_t net_conv3(const float* in, int cin, const float* w, const float* b, float* out, int cout, int H,
                            int W, int relu, const float* mask, hipStream_t s) {
  const unsigned gx = (unsigned)((W + kNT - 1) / kNT), gy = (unsigned)((H + kNT - 1) / kNT);
  if (cout % 8 == 0)
    hipLaunchKernelGGL(k_net_conv3<8>, dim3(gx, gy, (unsigned)(cout / 8)), dim3(256), 0, s, in, cin, w, b, out, cout,
                       H, W, relu, mask);
  else
    hipLaunchKernelGGL(k_net_conv3<2>, dim3(gx, gy, (unsigned)((cout + 1) / 2)), dim3(256), 0, s, in, cin, w, b, out,
                       cout, H, W, relu, mask);
  return hipGetLastError();
}

// ------------------------------------------------ inference on bfloat16 MFMA
// The predictor's forward pass, one layer per launch, as implicit GEMMs on
// v_mfma_f32_32x32x16_bf16: for a row segment of 32 pixels,
//   out[co][pixel] = b[co] + sum_k Wk[co][k] X[k][pixel],
// k = tap * CP + ci (tap = 3 ky + kx, channels padded to CP = 8 or 32), K
// padded to a multiple of 16 with zero weights, output channels padded to 32
// with zero weights.  Weights and activations are rounded to bfloat16 (RNE);
// products accumulate in float32; activations stay float32 in HBM.  A
// workgroup stages a 16 x 32 pixel tile plus a one-pixel circular halo in LDS
// as bfloat16, pixel-major with CP channels per pixel, so a lane's eight
// consecutive k are one 16-byte LDS read (the B operand); each wave holds the
// layer's whole weight matrix in registers (the A operand: lane l has output
// channel l % 32, k = 16 s + 8 (l / 32) .. +7 of step s) and computes 4 rows.
constexpr int kMR = 16;  // tile rows (4 per wave)
constexpr int kMC = 32;  // tile columns: one MFMA column block

template <int CP>
struct MfmaGeom {
  static constexpr int KP = ((9 * CP + 15) / 16) * 16;  // padded reduction length
  static constexpr int NS = KP / 16;                      // MFMA steps
};

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// wb[co][k] = bf16(w[co][ci][ky][kx]) for co < cout, tap = 3 ky + kx < 9,
// ci < cin (k = tap CP + ci); zero elsewhere; 32 rows of KP.
__global__ void k_net_pack_bf16(const float* __restrict__ w, int cin, int cout, int CP, int KP,
                                uint16_t* __restrict__ wb) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 32 * KP) return;
  const int co = idx / KP, k = idx - (idx / KP) * KP;
  const int tap = k / CP, ci = k - (k / CP) * CP;
  const float v = (co < cout && tap < 9 && ci < cin) ? w[((int64_t)co * cin + ci) * 9 + tap] : 0.0f;
  wb[idx] = (uint16_t)bf16_rne_bits(v);
}

// IN_BF: the input is the previous layer's bfloat16 output, pixel-major with
// 32 channels per pixel (else float32 channel-major images, converted while
// staged).  OUT_BF: the output is written that way for the next layer (else
// float32 channel-major images).  Bias and ReLU are applied in float32 before
// the rounding, so the values match rounding at the next layer's input.
// LDS slot of channel octet o of staged pixel pix.  With 32 channels a
// pixel takes 64 bytes, so the B fragments of 16 neighbouring pixels (one
// 16-byte read per lane) would share a quarter of the banks; the octet is
// XOR-swizzled with bits 2-3 of the pixel index, which puts 16 consecutive
// pixels on 16 distinct 16-byte bank groups.
template <int CP>
__device__ __forceinline__ int net_lds_off(int pix, int o) {
  if constexpr (CP == 32) return pix * CP + 8 * (o ^ ((pix >> 2) & 3));
  return pix * CP + 8 * o;
}

template <int CP, bool IN_BF, bool OUT_BF>
__global__ __launch_bounds__(256) void k_net_conv3_mfma(const void* __restrict__ in_, int cin,
                                                        const uint16_t* __restrict__ wb, const float* __restrict__ b,
                                                        void* __restrict__ out_, int cout, int H, int W, int relu) {
  using G = MfmaGeom<CP>;
  constexpr int SW = kMC + 2, NPIX = (kMR + 2) * SW, NOCT = CP / 8, ITEMS = NPIX * NOCT;
  __shared__ __align__(16) uint16_t s_x[NPIX * CP];
  // per-wave staging of one output row (32 pixels x 32 channels) so that the
  // bfloat16 output leaves as contiguous 16-byte stores
  __shared__ __align__(16) uint16_t s_o[OUT_BF ? 4 : 1][OUT_BF ? kMC * 32 : 8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v0 = blockIdx.x * kMC, u0 = blockIdx.y * kMR;
  const int64_t HW = (int64_t)H * W;
  uint4 a[G::NS];
#pragma unroll
  for (int st = 0; st < G::NS; ++st)
    a[st] = *reinterpret_cast<const uint4*>(wb + (lane & 31) * G::KP + 16 * st + 8 * (lane >> 5));
  // stage: each item is one pixel's octet of channels (one 16-byte LDS store);
  // items go in groups of 5 per thread with all their loads issued first
  constexpr int PER = (ITEMS + kThreads - 1) / kThreads, GRP = 5;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += GRP) {
    uint4 vals[GRP];
#pragma unroll
    for (int k = 0; k < GRP; ++k) {
      const int e = threadIdx.x + (k0 + k) * kThreads;
      if (k0 + k < PER && e < ITEMS) {
        // consecutive threads take consecutive octets of a pixel, so a wave
        // reads contiguous 16-byte pieces of the pixel-major rows
        const int pix = e / NOCT, o = e - (e / NOCT) * NOCT;
        const int i = pix / SW, j = pix - (pix / SW) * SW;
        const int64_t src = (int64_t)nwrap(u0 + i - 1, H) * W + nwrap(v0 + j - 1, W);
        if constexpr (IN_BF) {
          vals[k] = reinterpret_cast<const uint4*>(in_)[src * NOCT + o];
        } else {
          const float* in = static_cast<const float*>(in_);
          uint32_t wd[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c0 = 8 * o + 2 * q;
            const uint32_t lo = c0 < cin ? bf16_rne_bits(in[(int64_t)c0 * HW + src]) : 0u;
            const uint32_t hi = c0 + 1 < cin ? bf16_rne_bits(in[(int64_t)(c0 + 1) * HW + src]) : 0u;
            wd[q] = lo | (hi << 16);
          }
          vals[k] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < GRP; ++k) {
      const int e = threadIdx.x + (k0 + k) * kThreads;
      if (k0 + k < PER && e < ITEMS) {
        const int pix = e / NOCT, o = e - (e / NOCT) * NOCT;
        *reinterpret_cast<uint4*>(s_x + net_lds_off<CP>(pix, o)) = vals[k];
      }
    }
  }
  __syncthreads();
  const int j = lane & 31, h = lane >> 5;
  const int v = v0 + j;
#pragma unroll 1
  for (int r = 0; r < kMR / 4; ++r) {
    const int i = wave * (kMR / 4) + r;  // tile row
    floatx16 acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
#pragma unroll
    for (int st = 0; st < G::NS; ++st) {
      const int k0 = 16 * st + 8 * h;
      int tap = k0 / CP;
      const int ci0 = k0 - tap * CP;
      if (tap >= 9) tap = 0;  // padding k: zero weights, any staged value
      const int ky = tap / 3, kx = tap - 3 * (tap / 3);
      const uint4 bx = *reinterpret_cast<const uint4*>(s_x + net_lds_off<CP>((i + ky) * SW + j + kx, ci0 / 8));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[st]),
                                                    __builtin_bit_cast(bf16x8, bx), acc, 0, 0, 0);
    }
    const int u = u0 + i;
    // row of the 32 x 32 result held in acc[q]: 8 (q / 4) + 4 h + q % 4
    if constexpr (OUT_BF) {
      uint16_t* so = s_o[wave];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        uint32_t wd[2];
#pragma unroll
        for (int hq = 0; hq < 2; ++hq) {
          uint32_t bits[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const int q = 4 * g + 2 * hq + t, co = 8 * g + 4 * h + 2 * hq + t;
            float o = co < cout ? acc[q] + b[co] : 0.0f;
            if (relu) o = fmaxf(o, 0.0f);
            bits[t] = bf16_rne_bits(o);
          }
          wd[hq] = bits[0] | (bits[1] << 16);
        }
        *reinterpret_cast<uint2*>(so + j * 32 + 8 * g + 4 * h) = make_uint2(wd[0], wd[1]);
      }
      __builtin_amdgcn_wave_barrier();
      if (u < H) {
        uint16_t* out = static_cast<uint16_t*>(out_);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int idx = lane + 64 * t, pix = idx >> 2, oct = idx & 3;  // 16-byte pieces of the row
          if (v0 + pix < W)
            *reinterpret_cast<uint4*>(out + ((int64_t)u * W + v0 + pix) * 32 + 8 * oct) =
                *reinterpret_cast<const uint4*>(so + pix * 32 + 8 * oct);
        }
      }
      __builtin_amdgcn_wave_barrier();
    } else if (u < H && v < W) {
      const int64_t pxo = (int64_t)u * W + v;
      {
        float* out = static_cast<float*>(out_);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int co = 8 * (q >> 2) + 4 * h + (q & 3);
          if (co < cout) {
            float o = acc[q] + b[co];
            if (relu) o = fmaxf(o, 0.0f);
            out[(int64_t)co * HW + pxo] = o;
          }
        }
      }
    }
  }
}

// wt[ci][co][ky][kx] = w[co][ci][2-ky][2-kx]: the backward data pass is the
// forward convolution with these weights (cout and cin swapped).
__global__ void k_net_flip(const float* __restrict__ w, int cin, int cout, float* __restrict__ wt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cin * cout * 9) return;
  const int ci = e / (cout * 9), r = e - ci * cout * 9;
  const int co = r / 9, t = r - co * 9;
  const int ky = t / 3, kx = t - ky * 3;
  wt[e] = w[((int64_t)co * cin + ci) * 9 + (2 - ky) * 3 + (2 - kx)];
}

// Weight and bias gradients of one layer, partial sums per block:
// gw[co][ci][ky][kx] = sum_p g[co][p] in[ci][p + (ky-1, kx-1)], gb[co] = sum_p g[co][p].
// Block b takes pixel tiles b, b + gridDim.x, ...; thread t owns entries
// t, t + 256, ... of the layer's parameter vector (weights, then biases).
__global__ __launch_bounds__(256) void k_net_wgrad(const float* __restrict__ in, int cin, const float* __restrict__ g,
                                                   int cout, int H, int W, float* __restrict__ partials) {
  __shared__ float s_in[kNetMaxC * kNHalo * kNHalo];
  __shared__ float s_g[kNetMaxC * kNT * kNT];
  constexpr int kMaxPerThread = (kNetMaxC * kNetMaxC * 9 + kNetMaxC + 255) / 256;  // 37
  const int nw = cout * cin * 9, ne = nw + cout;
  const int64_t HW = (int64_t)H * W;
  const int tilesX = (W + kNT - 1) / kNT, tilesY = (H + kNT - 1) / kNT;
  float acc[kMaxPerThread];
#pragma unroll
  for (int k = 0; k < kMaxPerThread; ++k) acc[k] = 0.0f;
  for (int tile = blockIdx.x; tile < tilesX * tilesY; tile += gridDim.x) {
    const int u0 = (tile / tilesX) * kNT, v0 = (tile % tilesX) * kNT;
    __syncthreads();
    for (int e = threadIdx.x; e < cin * kNHalo * kNHalo; e += blockDim.x) {
      const int ci = e / (kNHalo * kNHalo), r = e - ci * (kNHalo * kNHalo);
      const int i = r / kNHalo, j = r - i * kNHalo;
      s_in[e] = in[(int64_t)ci * HW + (int64_t)nwrap(u0 + i - 1, H) * W + nwrap(v0 + j - 1, W)];
    }
    for (int e = threadIdx.x; e < cout * kNT * kNT; e += blockDim.x) {
      const int co = e / (kNT * kNT), r = e - co * kNT * kNT;
      const int u = u0 + r / kNT, v = v0 + r % kNT;
      s_g[e] = (u < H && v < W) ? g[(int64_t)co * HW + (int64_t)u * W + v] : 0.0f;  // outside: no contribution
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxPerThread; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e >= ne) break;
      float a = 0.0f;
      if (e < nw) {
        const int co = e / (cin * 9), r = e - co * cin * 9;
        const int ci = r / 9, t = r - ci * 9;
        const int ky = t / 3, kx = t - ky * 3;
        const float* gi = s_g + co * kNT * kNT;
        const float* xi = s_in + ci * kNHalo * kNHalo + ky * kNHalo + kx;
        for (int i = 0; i < kNT; ++i)
#pragma unroll 4
          for (int j = 0; j < kNT; ++j) a = fmaf(gi[i * kNT + j], xi[i * kNHalo + j], a);
      } else {
        const float* gi = s_g + (e - nw) * kNT * kNT;
        for (int i = 0; i < kNT * kNT; ++i) a += gi[i];
      }
      acc[k] += a;
    }
  }
#pragma unroll
  for (int k = 0; k < kMaxPerThread; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < ne) partials[(int64_t)blockIdx.x * ne + e] = acc[k];
  }
}

// out[e] = sum_b partials[b * n + e] in block order (double sums).
__global__ void k_net_sum_partials(const float* __restrict__ partials, int nblk, int n, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double a = 0.0;
  for (int b = 0; b < nblk; ++b) a += (double)partials[(int64_t)b * n + e];
  out[e] = (float)a;
}

// ------------------------------------------------ loss and its gradient
// Block partial sums of v over [0, n) into part[blockIdx.x] (double).
__device__ __forceinline__ void net_block_partial(double v, double* part) {
  __shared__ double shm[8];
  const double t = block_sum(v, shm);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[0] = sum of part[0..n): one block of 256 threads, thread t summing
// part[t], part[t + 256], ... in order, then a fixed-shape block reduction
// (deterministic; every load in flight at once instead of a serial chain)
__global__ __launch_bounds__(256) void k_net_finish_sum(const double* __restrict__ part, int n,
                                                        double* __restrict__ out) {
  __shared__ double shm[8];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a += part[i];
  const double t = block_sum(a, shm);
  if (threadIdx.x == 0) out[0] = t;
}

// Block partials of the loss normalisers: sum (mu_prev - mu_t)^2 into part,
// sum mu_t^2 into part + nblk, sum tgt^2 into part + 2 nblk, with
// tgt = log(clip(s_t d, 0.05, 20) / sb).
__global__ __launch_bounds__(256) void k_net_loss_norms(const float* __restrict__ aux, const float* __restrict__ tgt,
                                                        int64_t HW, double* __restrict__ part) {
  double a = 0.0, m = 0.0, t = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += (int64_t)gridDim.x * blockDim.x) {
    const double mp = aux[p], d = aux[HW + p], sb = aux[2 * HW + p];
    const double mt = tgt[p], st = tgt[HW + p];
    double sd = st * d;
    sd = sd < 0.05 ? 0.05 : (sd > 20.0 ? 20.0 : sd);
    const double lt = log(sd / sb);
    a += (mp - mt) * (mp - mt);
    m += mt * mt;
    t += lt * lt;
  }
  net_block_partial(a, part);
  net_block_partial(m, part + gridDim.x);
  net_block_partial(t, part + 2 * gridDim.x);
}

// nrm[0] = sum (mu_prev - mu_t)^2 + f sum mu_t^2, nrm[1] = sum tgt^2 + f HW
// from the three finished sums s[0..2] (f = kNetNormFloor); one thread
__global__ void k_net_finish_norms(const double* __restrict__ s3, int64_t HW, double* __restrict__ nrm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = s3[0] + kNetNormFloor * s3[1];
  nrm[0] = a > 0.0 ? a : 1.0;
  nrm[1] = s3[2] + kNetNormFloor * (double)HW;
}

// g = dL/d(out) and block partials of L (the normalisers in nrm[0..1])
__global__ __launch_bounds__(256) void k_net_loss_grad(const float* __restrict__ out, const float* __restrict__ aux,
                                                       const float* __restrict__ tgt, int64_t HW,
                                                       const double* __restrict__ nrm, float* __restrict__ g,
                                                       double* __restrict__ part) {
  const double nr = nrm[0], nd = nrm[1];
  double a = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += (int64_t)gridDim.x * blockDim.x) {
    const double o0 = out[p], o1 = out[HW + p];
    const double mp = aux[p], d = aux[HW + p], sb = aux[2 * HW + p];
    const double mt = tgt[p], st = tgt[HW + p];
    const double th = tanh(o0);
    const double e = mp * (1.0 + th) - mt;
    double sd = st * d;
    sd = sd < 0.05 ? 0.05 : (sd > 20.0 ? 20.0 : sd);
    const double r = o1 - log(sd / sb);
    a += e * e / nr + kNetLambdaD * r * r / nd;
    g[p] = (float)(2.0 * e * mp * (1.0 - th * th) / nr);
    g[HW + p] = (float)(2.0 * kNetLambdaD * r / nd);
  }
  net_block_partial(a, part);
}

// Adam (Kingma & Ba 2015) on the flat parameter vector; step >= 1.
__global__ void k_net_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                           float* __restrict__ v, int64_t n, float lr, int step) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)step));
  const float vh = vi / (1.0f - powf(b2, (float)step));
  theta[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------ features and prediction
__global__ __launch_bounds__(256) void k_net_mu_sumsq(const double* __restrict__ mu, int64_t n,
                                                      double* __restrict__ part) {
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a += mu[i] * mu[i];
  net_block_partial(a, part);
}

__global__ void k_net_features(const float* __restrict__ alpha, const float* __restrict__ alpha_prev,
                               const double* __restrict__ mu,
                               const float* __restrict__ s, const float* __restrict__ taps, int ntaps, double beta,
                               int64_t HW, const double* __restrict__ musq, float* __restrict__ feats,
                               float* __restrict__ aux) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  const double bh = beta * taps_sq_sum(taps, ntaps);
  const double a = alpha[p], d = bh + a;
  double rms = sqrt(musq[0] / (double)HW);
  if (!(rms > 0.0)) rms = 1.0;
  double sd = (double)s[p] * d;
  sd = sd < 1e-3 ? 1e-3 : (sd > 1e3 ? 1e3 : sd);
  feats[p] = (float)(a / d);
  feats[HW + p] = (float)(mu[p] / rms);
  // the logs in float32 of the float64 ratios (the features are float32
  // network inputs; about one ulp from the float64 logs)
  feats[2 * HW + p] = logf((float)sd) / 3.0f;
  feats[3 * HW + p] = logf((float)(d / bh)) / 10.0f;
  float lr = logf((float)((bh + (double)alpha_prev[p]) / d));
  lr = lr < -10.0f ? -10.0f : (lr > 10.0f ? 10.0f : lr);
  feats[4 * HW + p] = lr / 10.0f;
  aux[p] = (float)mu[p];
  aux[HW + p] = (float)d;
  double sb = (double)s[p] * d;
  sb = sb < 0.05 ? 0.05 : (sb > 20.0 ? 20.0 : sb);
  aux[2 * HW + p] = (float)sb;
}

// mu0 = mu_prev (1 + tanh o0) (float64, from the exact previous mean), d0 = exp(clip(o1)) sb / d
__global__ void k_net_predict(const float* __restrict__ out, const double* __restrict__ mu_prev,
                              const float* __restrict__ aux, int64_t HW, float* __restrict__ d0,
                              double* __restrict__ mu0) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  const double o0 = out[p];
  double o1 = out[HW + p];
  o1 = o1 < -10.0 ? -10.0 : (o1 > 10.0 ? 10.0 : o1);
  mu0[p] = mu_prev[p] * (1.0 + tanh(o0));
  d0[p] = (float)(exp(o1) * (double)aux[2 * HW + p] / (double)aux[HW + p]);
}

}  // namespace cofem

using namespace cofem;

struct cofem_net {
  int H = 0, W = 0;
  int64_t HW = 0, np = 0;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  float* act[kNetLayers + 1] = {};  // act[0] = features, act[4] = output
  float *g0 = nullptr, *g1 = nullptr, *wt = nullptr, *wpart = nullptr;
  float *feats = nullptr, *aux = nullptr;  // predictor scratch
  uint16_t* wbf = nullptr;                 // bfloat16 weights of the MFMA forward pass
  bool wbf_ok = false;                     // wbf holds the current theta (cleared where theta changes)
  hipEvent_t ev_pack = nullptr;            // end of the last packing of wbf ...
  hipStream_t pack_stream = nullptr;       // ... on this stream
  uint16_t* actb[2] = {};                  // its bfloat16 activations, pixel-major, 32 channels
  double *dpart = nullptr, *dscal = nullptr;
  int step = 0;
  int nred = 0;  // blocks of the reductions
};

namespace {

cofem_status net_fail(cofem_status s, const std::string& msg) {
  cofem::set_last_error(msg);
  return s;
}

#define NET_HIP(call)                                                                                      \
  do {                                                                                                     \
    hipError_t e_ = (call);                                                                                \
    if (e_ != hipSuccess)                                                                                  \
      return net_fail(e_ == hipErrorOutOfMemory ? COFEM_ERR_OUT_OF_MEMORY : COFEM_ERR_DEVICE,               \
                      std::string(#call) + ": " + hipGetErrorString(e_));                                  \
  } while (0)

template <typename T>
cofem_status net_alloc(cofem_net* n, T** p, size_t count) {
  void* q = nullptr;
  const size_t bytes = (count == 0 ? 1 : count) * sizeof(T);
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return net_fail(COFEM_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  n->allocs.push_back(q);
  *p = static_cast<T*>(q);
  NET_HIP(hipMemsetAsync(q, 0, bytes, n->stream));
  return COFEM_OK;
}

void net_free(cofem_net* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  if (n->ev_pack) {
    (void)hipEventSynchronize(n->ev_pack);
    (void)hipEventDestroy(n->ev_pack);
  }
  for (void* p : n->allocs) (void)hipFree(p);
  delete n;
}

int64_t layer_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += net_layer_params(i);
  return o;
}

// He-normal initial weights (std sqrt(2 / (9 cin))), zero biases, and a
// last layer of zeros: the untrained network predicts the previous mean and
// the previous diagonal estimate (clipped).  Normals from a counter-based SplitMix64 stream
// (Box-Muller), seeded by `seed`.
void net_init_host(std::vector<float>& th, uint64_t seed) {
  uint64_t ctr = 0;
  auto next = [&]() {
    uint64_t z = seed + (++ctr) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);  // (0, 1)
  };
  int64_t k = 0;
  for (int l = 0; l < kNetLayers; ++l) {
    const int ci = kNetCh[l], co = kNetCh[l + 1];
    const double sd = (l + 1 < kNetLayers) ? sqrt(2.0 / (9.0 * ci)) : 0.0;
    for (int64_t i = 0; i < (int64_t)co * ci * 9; ++i) {
      const double u1 = next(), u2 = next();
      th[k++] = (float)(sd * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    }
    for (int i = 0; i < co; ++i) th[k++] = 0.0f;
  }
}

cofem_status net_forward_impl(cofem_net* n, const float* feats) {
  const float* x = feats;
  for (int l = 0; l < kNetLayers; ++l) {
    const int64_t o = layer_offset(l);
    const float* w = n->theta + o;
    const float* b = w + (int64_t)kNetCh[l + 1] * kNetCh[l] * 9;
    NET_HIP(net_conv3(x, kNetCh[l], w, b, n->act[l + 1], kNetCh[l + 1], n->H, n->W, l + 1 < kNetLayers ? 1 : 0,
                      nullptr, n->stream));
    x = n->act[l + 1];
  }
  return COFEM_OK;
}

// The forward pass on bfloat16 MFMA (inference): the weights packed per
// layer when theta has changed since the last packing, then one
// implicit-GEMM launch per layer into act[1..4].
cofem_status net_forward_bf16_impl(cofem_net* n, const float* feats) {
  auto layer_kp = [](int l) { return l == 0 ? MfmaGeom<8>::KP : MfmaGeom<32>::KP; };
  if (!n->wbf_ok) {
    int64_t off = 0;
    for (int l = 0; l < kNetLayers; ++l) {
      const int ci = kNetCh[l], co = kNetCh[l + 1], KP = layer_kp(l);
      hipLaunchKernelGGL(k_net_pack_bf16, dim3((unsigned)((32 * KP + 255) / 256)), dim3(256), 0, n->stream,
                         n->theta + layer_offset(l), ci, co, l == 0 ? 8 : 32, KP, n->wbf + off);
      off += 32 * KP;
    }
    NET_HIP(hipGetLastError());
    if (!n->ev_pack) NET_HIP(hipEventCreateWithFlags(&n->ev_pack, hipEventDisableTiming));
    NET_HIP(hipEventRecord(n->ev_pack, n->stream));
    n->pack_stream = n->stream;
    n->wbf_ok = true;
  } else if (n->stream != n->pack_stream) {
    NET_HIP(hipStreamWaitEvent(n->stream, n->ev_pack, 0));
  }
  int64_t off = 0;
  const dim3 grid((unsigned)((n->W + kMC - 1) / kMC), (unsigned)((n->H + kMR - 1) / kMR));
  for (int l = 0; l < kNetLayers; ++l) {
    const int ci = kNetCh[l], co = kNetCh[l + 1];
    const float* bias = n->theta + layer_offset(l) + (int64_t)co * ci * 9;
    const uint16_t* wb = n->wbf + off;
    off += 32 * layer_kp(l);
    // layer 0: float32 features -> bf16 act; 1, 2: bf16 -> bf16; 3: bf16 -> float32 output
    uint16_t* ping = n->actb[l & 1];
    const uint16_t* pong = n->actb[(l + 1) & 1];
    if (l == 0)
      hipLaunchKernelGGL((k_net_conv3_mfma<8, false, true>), grid, dim3(256), 0, n->stream, feats, ci, wb, bias, ping,
                         co, n->H, n->W, 1);
    else if (l + 1 < kNetLayers)
      hipLaunchKernelGGL((k_net_conv3_mfma<32, true, true>), grid, dim3(256), 0, n->stream, pong, ci, wb, bias, ping,
                         co, n->H, n->W, 1);
    else
      hipLaunchKernelGGL((k_net_conv3_mfma<32, true, false>), grid, dim3(256), 0, n->stream, pong, ci, wb, bias,
                         n->act[kNetLayers], co, n->H, n->W, 0);
    NET_HIP(hipGetLastError());
  }
  return COFEM_OK;
}

// forward, loss and all parameter gradients into n->grad; loss into dscal[1]
cofem_status net_loss_grad_impl(cofem_net* n, const float* feats, const float* aux, const float* tgt) {
  if (cofem_status s = net_forward_impl(n, feats)) return s;
  const int nb = n->nred;
  // dscal: [1] loss, [3..5] the three normaliser sums, [6..7] the normalisers
  hipLaunchKernelGGL(k_net_loss_norms, dim3(nb), dim3(256), 0, n->stream, aux, tgt, n->HW, n->dpart);
  for (int i = 0; i < 3; ++i)
    hipLaunchKernelGGL(k_net_finish_sum, dim3(1), dim3(256), 0, n->stream, n->dpart + i * nb, nb, n->dscal + 3 + i);
  hipLaunchKernelGGL(k_net_finish_norms, dim3(1), dim3(64), 0, n->stream, n->dscal + 3, n->HW, n->dscal + 6);
  hipLaunchKernelGGL(k_net_loss_grad, dim3(nb), dim3(256), 0, n->stream, n->act[kNetLayers], aux, tgt, n->HW,
                     n->dscal + 6, n->g0, n->dpart);
  hipLaunchKernelGGL(k_net_finish_sum, dim3(1), dim3(256), 0, n->stream, n->dpart, nb, n->dscal + 1);
  NET_HIP(hipGetLastError());
  float* g = n->g0;
  float* gn = n->g1;
  for (int l = kNetLayers - 1; l >= 0; --l) {
    const int ci = kNetCh[l], co = kNetCh[l + 1];
    const float* x = l == 0 ? feats : n->act[l];
    const int64_t o = layer_offset(l);
    const int ne = co * ci * 9 + co;
    hipLaunchKernelGGL(k_net_wgrad, dim3(kNetWgBlocks), dim3(256), 0, n->stream, x, ci, g, co, n->H, n->W, n->wpart);
    hipLaunchKernelGGL(k_net_sum_partials, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, n->stream, n->wpart,
                       kNetWgBlocks, ne, n->grad + o);
    NET_HIP(hipGetLastError());
    if (l > 0) {
      hipLaunchKernelGGL(k_net_flip, dim3((unsigned)((ci * co * 9 + 255) / 256)), dim3(256), 0, n->stream,
                         n->theta + o, ci, co, n->wt);
      // gradient w.r.t. this layer's input, through the ReLU of the layer below
      NET_HIP(net_conv3(g, co, n->wt, nullptr, gn, ci, n->H, n->W, 0, n->act[l], n->stream));
      float* t = g;
      g = gn;
      gn = t;
    }
  }
  return COFEM_OK;
}

}  // namespace

namespace cofem {

// Predictor of the learned form: from the solver state (alpha, the previous
// float64 mean and the previous diagonal estimate) fills the probe columns'
// start scale d0 and the mean start mu0 for the next E-step.
cofem_status net_predict(cofem_net* n, const float* alpha, const float* alpha_prev, const double* mu_prev,
                         const float* s_prev, const float* taps, int ntaps, double beta, float* d0, double* mu0,
                         hipStream_t s) {
  const int nb = n->nred;
  hipLaunchKernelGGL(k_net_mu_sumsq, dim3(nb), dim3(256), 0, s, mu_prev, n->HW, n->dpart);
  hipLaunchKernelGGL(k_net_finish_sum, dim3(1), dim3(256), 0, s, n->dpart, nb, n->dscal + 2);
  const unsigned g = (unsigned)((n->HW + 255) / 256);
  hipLaunchKernelGGL(k_net_features, dim3(g), dim3(256), 0, s, alpha, alpha_prev, mu_prev, s_prev, taps, ntaps, beta,
                     n->HW, n->dscal + 2, n->feats, n->aux);
  NET_HIP(hipGetLastError());
  hipStream_t keep = n->stream;
  n->stream = s;
  const cofem_status st = net_forward_bf16_impl(n, n->feats);
  n->stream = keep;
  if (st != COFEM_OK) return st;
  hipLaunchKernelGGL(k_net_predict, dim3(g), dim3(256), 0, s, n->act[kNetLayers], mu_prev, n->aux, n->HW, d0, mu0);
  NET_HIP(hipGetLastError());
  return COFEM_OK;
}

cofem_status net_features(cofem_net* n, const float* alpha, const float* alpha_prev, const double* mu_prev,
                          const float* s_prev, const float* taps, int ntaps, double beta, float* feats, float* aux,
                          hipStream_t s) {
  const int nb = n->nred;
  hipLaunchKernelGGL(k_net_mu_sumsq, dim3(nb), dim3(256), 0, s, mu_prev, n->HW, n->dpart);
  hipLaunchKernelGGL(k_net_finish_sum, dim3(1), dim3(256), 0, s, n->dpart, nb, n->dscal + 2);
  hipLaunchKernelGGL(k_net_features, dim3((unsigned)((n->HW + 255) / 256)), dim3(256), 0, s, alpha, alpha_prev,
                     mu_prev, s_prev, taps, ntaps, beta, n->HW, n->dscal + 2, feats, aux);
  NET_HIP(hipGetLastError());
  return COFEM_OK;
}

int net_height(const cofem_net* n) { return n->H; }
int net_width(const cofem_net* n) { return n->W; }

}  // namespace cofem

extern "C" {

int64_t cofem_net_num_params(void) {
  int64_t t = 0;
  for (int l = 0; l < kNetLayers; ++l) t += net_layer_params(l);
  return t;
}

cofem_status cofem_net_create(int32_t H, int32_t W, uint64_t seed, void* hip_stream, cofem_net** out) {
  if (!out) return net_fail(COFEM_ERR_INVALID_ARG, "out is null");
  if (H < 1 || W < 1 || (int64_t)H * W > (int64_t)1 << 26) return net_fail(COFEM_ERR_INVALID_ARG, "bad image size");
  cofem_net* n = new (std::nothrow) cofem_net();
  if (!n) return net_fail(COFEM_ERR_OUT_OF_MEMORY, "host allocation failed");
  n->H = H;
  n->W = W;
  n->HW = (int64_t)H * W;
  n->np = cofem_net_num_params();
  n->stream = static_cast<hipStream_t>(hip_stream);
  n->nred = (int)((n->HW + 4 * 256 - 1) / (4 * 256));
  if (n->nred > 1024) n->nred = 1024;
  cofem_status s = COFEM_OK;
  auto A = [&](auto** p, size_t c) {
    if (s == COFEM_OK) s = net_alloc(n, p, c);
  };
  A(&n->theta, (size_t)n->np);
  A(&n->grad, (size_t)n->np);
  A(&n->m, (size_t)n->np);
  A(&n->v, (size_t)n->np);
  for (int l = 1; l <= kNetLayers; ++l) A(&n->act[l], (size_t)kNetCh[l] * n->HW);
  A(&n->g0, (size_t)kNetMaxC * n->HW);
  A(&n->g1, (size_t)kNetMaxC * n->HW);
  A(&n->wt, (size_t)kNetMaxC * kNetMaxC * 9);
  A(&n->wpart, (size_t)kNetWgBlocks * (kNetMaxC * kNetMaxC * 9 + kNetMaxC));
  A(&n->feats, (size_t)kNetCh[0] * n->HW);
  A(&n->aux, (size_t)3 * n->HW);
  A(&n->wbf, (size_t)32 * (MfmaGeom<8>::KP + (kNetLayers - 1) * MfmaGeom<32>::KP));
  A(&n->actb[0], (size_t)32 * n->HW);
  A(&n->actb[1], (size_t)32 * n->HW);
  A(&n->dpart, (size_t)3 * n->nred);
  A(&n->dscal, 8);
  if (s == COFEM_OK) {
    std::vector<float> th((size_t)n->np);
    net_init_host(th, seed);
    hipError_t e = hipMemcpyAsync(n->theta, th.data(), sizeof(float) * th.size(), hipMemcpyHostToDevice, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) s = net_fail(COFEM_ERR_DEVICE, std::string("net init: ") + hipGetErrorString(e));
  }
  if (s != COFEM_OK) {
    net_free(n);
    return s;
  }
  *out = n;
  return COFEM_OK;
}

void cofem_net_destroy(cofem_net* net) { net_free(net); }

cofem_status cofem_net_set_params(cofem_net* n, const float* host_params, int64_t count) {
  if (!n || !host_params || count != n->np) return net_fail(COFEM_ERR_INVALID_ARG, "bad net, pointer or count");
  NET_HIP(hipMemcpyAsync(n->theta, host_params, sizeof(float) * count, hipMemcpyHostToDevice, n->stream));
  NET_HIP(hipMemsetAsync(n->m, 0, sizeof(float) * count, n->stream));
  NET_HIP(hipMemsetAsync(n->v, 0, sizeof(float) * count, n->stream));
  NET_HIP(hipStreamSynchronize(n->stream));
  n->step = 0;
  n->wbf_ok = false;
  return COFEM_OK;
}

cofem_status cofem_net_get_params(cofem_net* n, float* host_params, int64_t count) {
  if (!n || !host_params || count != n->np) return net_fail(COFEM_ERR_INVALID_ARG, "bad net, pointer or count");
  NET_HIP(hipMemcpyAsync(host_params, n->theta, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
  NET_HIP(hipStreamSynchronize(n->stream));
  return COFEM_OK;
}

cofem_status cofem_net_forward(cofem_net* n, const float* feats, float* out) {
  if (!n || !feats || !out) return net_fail(COFEM_ERR_INVALID_ARG, "null argument");
  if (cofem_status s = net_forward_impl(n, feats)) return s;
  NET_HIP(hipMemcpyAsync(out, n->act[kNetLayers], sizeof(float) * 2 * n->HW, hipMemcpyDeviceToDevice, n->stream));
  NET_HIP(hipStreamSynchronize(n->stream));
  return COFEM_OK;
}

cofem_status cofem_net_forward_bf16(cofem_net* n, const float* feats, float* out) {
  if (!n || !feats || !out) return net_fail(COFEM_ERR_INVALID_ARG, "null argument");
  if (cofem_status s = net_forward_bf16_impl(n, feats)) return s;
  NET_HIP(hipMemcpyAsync(out, n->act[kNetLayers], sizeof(float) * 2 * n->HW, hipMemcpyDeviceToDevice, n->stream));
  NET_HIP(hipStreamSynchronize(n->stream));
  return COFEM_OK;
}

cofem_status cofem_net_loss_grad(cofem_net* n, const float* feats, const float* aux, const float* targets,
                                 double* loss, float* host_grad) {
  if (!n || !feats || !aux || !targets) return net_fail(COFEM_ERR_INVALID_ARG, "null argument");
  if (cofem_status s = net_loss_grad_impl(n, feats, aux, targets)) return s;
  if (loss) NET_HIP(hipMemcpyAsync(loss, n->dscal + 1, sizeof(double), hipMemcpyDeviceToHost, n->stream));
  if (host_grad)
    NET_HIP(hipMemcpyAsync(host_grad, n->grad, sizeof(float) * n->np, hipMemcpyDeviceToHost, n->stream));
  NET_HIP(hipStreamSynchronize(n->stream));
  return COFEM_OK;
}

cofem_status cofem_net_train_step(cofem_net* n, const float* feats, const float* aux, const float* targets, float lr,
                                  double* loss) {
  if (!n || !feats || !aux || !targets) return net_fail(COFEM_ERR_INVALID_ARG, "null argument");
  if (!(lr > 0.0f)) return net_fail(COFEM_ERR_INVALID_ARG, "lr must be positive");
  if (cofem_status s = net_loss_grad_impl(n, feats, aux, targets)) return s;
  ++n->step;
  hipLaunchKernelGGL(k_net_adam, dim3((unsigned)((n->np + 255) / 256)), dim3(256), 0, n->stream, n->theta, n->grad,
                     n->m, n->v, n->np, lr, n->step);
  NET_HIP(hipGetLastError());
  n->wbf_ok = false;
  if (loss) {
    NET_HIP(hipMemcpyAsync(loss, n->dscal + 1, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    NET_HIP(hipStreamSynchronize(n->stream));
  }
  return COFEM_OK;
}

}  // extern "C"
