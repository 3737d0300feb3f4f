// The two stencil stages of the convolution dictionary's operator pass on one
// output tile, shared by the per-tile kernels (kernels_conv.hip) and the
// persistent warp-specialised kernel (kernels_conv_ws.hip).
//
// Phi is a circular convolution with an odd KS x KS kernel h, c = (KS-1)/2:
//   (Phi z)[u, v]   = sum_{a,b} h[a,b] z[(u - a + c) mod H, (v - b + c) mod W]
//   (Phi^T w)[u, v] = sum_{a,b} h[a,b] w[(u + a - c) mod H, (v + b - c) mod W]
// Stage 1 forms t = Phi p on a TILE x TILE tile plus a c halo from p staged
// in LDS with a 2c halo; stage 2 forms Phi^T t on the tile.  Each thread
// computes 4x4 output blocks.
#pragma once

#include "cofem_internal.h"

namespace cofem {

__device__ __forceinline__ int wrap(int x, int n) {
  x %= n;
  return x < 0 ? x + n : x;
}

// Geometry of one pass over a TILE x TILE output tile with KS x KS taps.
// Stage 1 forms t on the tile plus a c halo (TR x TR, rounded up to 4x4
// blocks) from p staged with a 2c halo (SPH x SPW); a 4x4 block reads KS+3
// rows of XW values (KS+3 rounded up to whole float4s).
template <int KS, int TILE>
struct ConvGeom {
  static constexpr int c = (KS - 1) / 2;
  static constexpr int TR = ((TILE + 2 * c + 3) / 4) * 4;
  static constexpr int XW = ((KS + 3 + 3) / 4) * 4;
  static constexpr int SPH = TR + 2 * c;
  static constexpr int SPW = TR + XW - 4;
  static constexpr int NB1 = (TR / 4) * (TR / 4);
  static constexpr int NB2 = (TILE / 4) * (TILE / 4);
  static constexpr int LDS = SPH * SPW + TR * TR;  // values
};

// Taps of the 4x4 blocks, read from LDS as broadcasts.  Each input row uses
// at most 4 tap rows (4 KS values), which stay in registers for that row;
// fence() is an empty asm that the compiler must assume changes the (zero)
// index offset, so tap reads of later rows are neither merged with nor
// hoisted above earlier ones (keeping all KS*KS taps live would crowd out the
// accumulators and the double-buffered input rows).
template <typename T>
struct Taps {
  typedef __attribute__((address_space(3))) const T* lds_ptr;
  lds_ptr s;     // the taps in LDS (an LDS-typed pointer, so reads stay ds_read)
  lds_ptr base;  // s laundered by fence(): one address register per input
                 // row, the row's tap reads use immediate offsets from it
  __device__ __forceinline__ explicit Taps(const T* p) : s((lds_ptr)p), base((lds_ptr)p) {}
  __device__ __forceinline__ T operator()(int i) const { return base[i]; }
  __device__ __forceinline__ void fence() {
    base = s;
    asm volatile("" : "+v"(base));
  }
};

// Taps held in registers (read from LDS once per use of the stencil stages):
// for a kernel whose stencil waves have registers to spare, it removes the
// per-row tap reads from their instruction stream.
template <int KS>
struct TapsReg {
  float v[KS * KS];
  __device__ __forceinline__ explicit TapsReg(const float* lds) {
#pragma unroll
    for (int i = 0; i < KS * KS; ++i) v[i] = lds[i];
  }
  __device__ __forceinline__ float operator()(int i) const { return v[i]; }
  __device__ __forceinline__ void fence() {}
};

template <typename T, int N>
__device__ __forceinline__ void lds_row(const T* src, T (&x)[N]) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int q = 0; q < N / 4; ++q) {
      const float4 v = reinterpret_cast<const float4*>(src)[q];
      x[4 * q] = v.x;
      x[4 * q + 1] = v.y;
      x[4 * q + 2] = v.z;
      x[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < N / 2; ++q) {
      const double2 v = reinterpret_cast<const double2*>(src)[q];
      x[2 * q] = v.x;
      x[2 * q + 1] = v.y;
    }
  }
}

// Stage 1 over the 4x4 blocks item = tid, tid + nthr, ...:
//   t(i, j) = sum_{a,b} h[a][b] sP(i - a + 2c, j - b + 2c)
// sP is SPH x SPW, sT is TR x TR.
template <int KS, int TILE, typename T, typename TapsT>
__device__ __forceinline__ void conv_stage1(TapsT h, const T* sP, T* sT, int tid, int nthr) {
  using G = ConvGeom<KS, TILE>;
  constexpr int c = G::c;
  for (int item = tid; item < G::NB1; item += nthr) {
    const int bi = item / (G::TR / 4), bj = item - (item / (G::TR / 4)) * (G::TR / 4);
    T acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) acc[r][cc] = T(0);
    // rows are double-buffered: row q + 1 is read from LDS while row q is
    // used; the scheduling barrier keeps later rows' loads from being hoisted
    // (which would hold every row in registers at once)
    const T* src1 = sP + (4 * bi) * G::SPW + 4 * bj;
    T x[2][G::XW];
    lds_row(src1, x[0]);
#pragma unroll
    for (int q = 0; q < KS + 3; ++q) {  // input row 4 bi + q
      h.fence();
      if (q + 1 < KS + 3) lds_row(src1 + (q + 1) * G::SPW, x[(q + 1) & 1]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = r + 2 * c - q;
        if (a < 0 || a >= KS) continue;
#pragma unroll
        for (int b = 0; b < KS; ++b) {
          const T hv = h(a * KS + b);
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) acc[r][cc] = fma(hv, x[q & 1][cc + 2 * c - b], acc[r][cc]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T* dst = sT + (4 * bi + r) * G::TR + 4 * bj;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) dst[cc] = acc[r][cc];
    }
  }
}

// Stage 1 in 4x6 blocks (float, TR a multiple of 6): TR/4 x TR/6 items,
// e.g. 216 for the 72 x 72 region of a 64 x 64 tile with 9x9 taps, one
// round of a 256-thread group instead of the 4x4 blocks' 324 (two rounds for
// some waves).  A block reads KS+3 rows of 6 + 2c values as float2s.
template <int KS, int TILE>
struct Stage1W6 {
  using G = ConvGeom<KS, TILE>;
  static constexpr bool ok = G::TR % 6 == 0;
  static constexpr int NB = (G::TR / 4) * (G::TR / 6);
  static constexpr int XW = ((6 + 2 * G::c) + 1) / 2 * 2;
};
template <int KS, int TILE, typename TapsT>
__device__ __forceinline__ void conv_stage1_w6(TapsT h, const float* sP, float* sT, int tid, int nthr) {
  using G = ConvGeom<KS, TILE>;
  using S = Stage1W6<KS, TILE>;
  static_assert(S::ok, "4x6 blocks need TR divisible by 6");
  constexpr int c = G::c, NBJ = G::TR / 6;
  for (int item = tid; item < S::NB; item += nthr) {
    const int bi = item / NBJ, bj = item - (item / NBJ) * NBJ;
    float acc[4][6];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int cc = 0; cc < 6; ++cc) acc[r][cc] = 0.0f;
    const float* src1 = sP + (4 * bi) * G::SPW + 6 * bj;
    float x[2][S::XW];
    auto row = [&](const float* src, float (&xr)[S::XW]) {
#pragma unroll
      for (int q = 0; q < S::XW / 2; ++q) {
        const float2 v = reinterpret_cast<const float2*>(src)[q];
        xr[2 * q] = v.x;
        xr[2 * q + 1] = v.y;
      }
    };
    row(src1, x[0]);
#pragma unroll
    for (int q = 0; q < KS + 3; ++q) {  // input row 4 bi + q
      h.fence();
      if (q + 1 < KS + 3) row(src1 + (q + 1) * G::SPW, x[(q + 1) & 1]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = r + 2 * c - q;
        if (a < 0 || a >= KS) continue;
#pragma unroll
        for (int b = 0; b < KS; ++b) {
          const float hv = h(a * KS + b);
#pragma unroll
          for (int cc = 0; cc < 6; ++cc) acc[r][cc] = fma(hv, x[q & 1][cc + 2 * c - b], acc[r][cc]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float2* dst = reinterpret_cast<float2*>(sT + (4 * bi + r) * G::TR + 6 * bj);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) dst[cc] = make_float2(acc[r][2 * cc], acc[r][2 * cc + 1]);
    }
  }
}

// Stage 2 for 4x4 block tid (< NB2) of the tile:
//   (Phi^T t)(i, j) = sum_{a,b} h[a][b] t(i + a, j + b)
template <int KS, int TILE, typename T, typename TapsT>
__device__ __forceinline__ void conv_stage2(TapsT h, const T* sT, int tid, T (&acc)[4][4]) {
  using G = ConvGeom<KS, TILE>;
  const int bi = tid / (TILE / 4), bj = tid - (tid / (TILE / 4)) * (TILE / 4);
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) acc[r][cc] = T(0);
  const T* src2 = sT + (4 * bi) * G::TR + 4 * bj;
  T x[2][G::XW];
  lds_row(src2, x[0]);
#pragma unroll
  for (int q = 0; q < KS + 3; ++q) {  // t row 4 bi + q
    h.fence();
    if (q + 1 < KS + 3) lds_row(src2 + (q + 1) * G::TR, x[(q + 1) & 1]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = q - r;
      if (a < 0 || a >= KS) continue;
#pragma unroll
      for (int b = 0; b < KS; ++b) {
        const T hv = h(a * KS + b);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) acc[r][cc] = fma(hv, x[q & 1][cc + b], acc[r][cc]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The stencil stages in BR x BC output blocks (any block shape that divides
// the region; used where the 4x4 blocks would leave waves idle, e.g. the
// 32 x 32 float64 quadrants: 100 stage-1 and 64 stage-2 blocks of 4x4 on four
// waves).  Each output's sum runs over the same (input row, tap column) order
// as in the 4x4 forms.  Rows of XW = BC + 2c values are read as 16-byte
// vectors (XW * sizeof(T) and the block origins 16-byte aligned).
template <int KS, int TILE, int BR, int BC, typename T>
struct StageBlk {
  using G = ConvGeom<KS, TILE>;
  static constexpr int c = G::c, XW = BC + 2 * c, NV = 16 / sizeof(T);
  static constexpr int NB1 = (G::TR / BR) * (G::TR / BC), NB2 = (TILE / BR) * (TILE / BC);
  static_assert(G::TR % BR == 0 && G::TR % BC == 0 && TILE % BR == 0 && TILE % BC == 0, "block divides region");
  static_assert(XW % NV == 0 && (BC * sizeof(T)) % 16 == 0, "16-byte rows");
};
template <typename T, int N>
__device__ __forceinline__ void lds_row_v(const T* src, T (&x)[N]) {
  constexpr int NV = 16 / sizeof(T);
#pragma unroll
  for (int q = 0; q < N / NV; ++q) {
    if constexpr (sizeof(T) == 4) {
      const float4 v = reinterpret_cast<const float4*>(src)[q];
      x[4 * q] = v.x;
      x[4 * q + 1] = v.y;
      x[4 * q + 2] = v.z;
      x[4 * q + 3] = v.w;
    } else {
      const double2 v = reinterpret_cast<const double2*>(src)[q];
      x[2 * q] = v.x;
      x[2 * q + 1] = v.y;
    }
  }
}
template <int KS, int TILE, int BR, int BC, typename T, typename TapsT>
__device__ __forceinline__ void conv_stage1_blk(TapsT h, const T* sP, T* sT, int tid, int nthr) {
  using G = ConvGeom<KS, TILE>;
  using S = StageBlk<KS, TILE, BR, BC, T>;
  constexpr int c = G::c, NBJ = G::TR / BC;
  for (int item = tid; item < S::NB1; item += nthr) {
    const int bi = item / NBJ, bj = item - (item / NBJ) * NBJ;
    T acc[BR][BC];
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int cc = 0; cc < BC; ++cc) acc[r][cc] = T(0);
    const T* src1 = sP + (BR * bi) * G::SPW + BC * bj;
    T x[2][S::XW];
    lds_row_v(src1, x[0]);
#pragma unroll
    for (int q = 0; q < KS + BR - 1; ++q) {  // input row BR bi + q
      h.fence();
      if (q + 1 < KS + BR - 1) lds_row_v(src1 + (q + 1) * G::SPW, x[(q + 1) & 1]);
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        const int a = r + 2 * c - q;
        if (a < 0 || a >= KS) continue;
#pragma unroll
        for (int b = 0; b < KS; ++b) {
          const T hv = h(a * KS + b);
#pragma unroll
          for (int cc = 0; cc < BC; ++cc) acc[r][cc] = fma(hv, x[q & 1][cc + 2 * c - b], acc[r][cc]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      T* dst = sT + (BR * bi + r) * G::TR + BC * bj;
#pragma unroll
      for (int cc = 0; cc < BC; ++cc) dst[cc] = acc[r][cc];
    }
  }
}
// Stage 2 for block `item` (< NB2) of the tile: acc = (Phi^T t) on the block.
template <int KS, int TILE, int BR, int BC, typename T, typename TapsT>
__device__ __forceinline__ void conv_stage2_blk(TapsT h, const T* sT, int item, T (&acc)[BR][BC]) {
  using G = ConvGeom<KS, TILE>;
  using S = StageBlk<KS, TILE, BR, BC, T>;
  constexpr int NBJ = TILE / BC;
  const int bi = item / NBJ, bj = item - (item / NBJ) * NBJ;
#pragma unroll
  for (int r = 0; r < BR; ++r)
#pragma unroll
    for (int cc = 0; cc < BC; ++cc) acc[r][cc] = T(0);
  const T* src2 = sT + (BR * bi) * G::TR + BC * bj;
  T x[2][S::XW];
  lds_row_v(src2, x[0]);
#pragma unroll
  for (int q = 0; q < KS + BR - 1; ++q) {  // t row BR bi + q
    h.fence();
    if (q + 1 < KS + BR - 1) lds_row_v(src2 + (q + 1) * G::TR, x[(q + 1) & 1]);
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int a = q - r;
      if (a < 0 || a >= KS) continue;
#pragma unroll
      for (int b = 0; b < KS; ++b) {
        const T hv = h(a * KS + b);
#pragma unroll
        for (int cc = 0; cc < BC; ++cc) acc[r][cc] = fma(hv, x[q & 1][cc + b], acc[r][cc]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

}  // namespace cofem
