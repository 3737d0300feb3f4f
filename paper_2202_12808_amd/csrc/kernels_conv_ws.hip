// Persistent, warp-specialised form of the convolution dictionary's fused CG
// iteration (the operator application q = beta Phi^T Phi p + alpha (.) p of
// Sec. 3.2 with the previous CG update folded in, as k_conv_fused computes it).
//
// A tile's work has a memory part (stage p with its halo while applying the
// update x += a p, r' = r - a q, z = M^-1 r', p' = z + b p; the epilogue
// q = beta Phi^T t + alpha p' with its dot products) and an arithmetic part
// (the two stencil stages, 2 KS^2 FMAs per pixel).  In the per-tile kernel a
// workgroup runs them one after the other; here each workgroup is persistent
// and splits its waves by role so the two parts of different tiles overlap:
//   compute waves (4): stage 1 and stage 2 of unit s (LDS only);
//   memory waves (8):  staging of unit s + 1 and the epilogue of unit s - 1.
// The staging keeps r' and M^-1 of the unit's own pixels in LDS beside p',
// so the epilogue reads only alpha from memory.  The schedule of one step
// (two barriers, the same count for every wave) is described at
// ws_compute_loop; the role functions contain no other barrier.
//
// Units: the 32 x 32 quadrants of the float64 mean columns first, then the
// 64 x 64 tiles of the float probe columns.  Unit u belongs to workgroup
// slot u mod G at step u / G; slots are numbered so that the workgroups of
// one XCD (blockIdx mod 8) hold a contiguous band of tiles, whose halos then
// meet in one L2.  A unit's five sums (r'^T z, r'^T r', gam, del, eta) go to
// the column's partial rows in unit order; the wave depositing a column's
// last unit sums the rows in a fixed order, and the last workgroup to finish
// takes the step's scalars from the column totals (finish_fused), so results
// do not depend on timing.
#include <type_traits>

#include "conv_tile.h"

namespace cofem {

namespace {

// What a launch computes (a template parameter):
//   kWsFused  the previous CG update folded into the operator pass (one CG
//             iteration after a solve's first);
//   kWsPass   the operator pass on p with the step's dots gam = p^T q,
//             del = r^T M^-1 q, eta = q^T M^-1 q (a solve's first iteration);
//   kWsApply  q = A p alone;
//   kWsInit   the start of a warm-started solve: with q = A x0, r = b - q and
//             z = M^-1 r written as the solve's R and P, and per column
//             r^T z, r^T r, b^T b (q itself is not stored);
//   kWsResid  the true residual after a solve: per column ||b - A x||^2
//             (nothing is stored).
// The last three stage p (x) alone; b is the probe (regenerated from its
// counter-based hash) or the mean column's b0.
constexpr int kWsFused = 0, kWsPass = 1, kWsApply = 2, kWsInit = 3, kWsResid = 4;

constexpr int kWsCompute = 256;  // compute threads (waves 0-3)
constexpr int kWsMemory = 512;   // memory threads (waves 4-11)
constexpr int kWsThreads = kWsCompute + kWsMemory;
constexpr int kWsMemWaves = kWsMemory / 64;

template <int KS>
struct WsGeom {
  using GF = ConvGeom<KS, kConvTile>;       // float tile
  using GD = ConvGeom<KS, kConvTile / 2>;   // float64 quadrant
  static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t SP = (mx(GF::SPH * GF::SPW * 4, GD::SPH * GD::SPW * 8) + 15) / 16 * 16;
  static constexpr size_t ST = (mx(GF::TR * GF::TR * 4, GD::TR * GD::TR * 8) + 15) / 16 * 16;
  // a unit's own pixels: Phi^T t (sU) and the staged r', M^-1 (sR, sM)
  static constexpr size_t SU = mx(kConvTile * kConvTile * 4, (kConvTile / 2) * (kConvTile / 2) * 8);
  // two staged regions, stage-1 output, stage-2 output, two r' and two M^-1
  static constexpr size_t BYTES = 2 * SP + ST + 5 * SU;
  static_assert(GF::SPW % 4 == 0 && GD::SPW % 2 == 0 && (2 * GF::c) % 4 == 0, "vector rows");
};

struct WsUnit {
  int col;       // column: probe (< K, float) or mean (>= K, float64)
  int blk;       // row of its sums in the column's partials (tile * nparts + part)
  int nblk;      // units of the column
  int tu0, tv0;  // output origin
  bool is64, inside, exists;
};

__device__ __forceinline__ WsUnit ws_unit(int u, int U, int ntiles, int tilesX, int K, int nt, int H, int W) {
  WsUnit x;
  x.exists = u >= 0 && u < U;
  x.col = 0;
  x.blk = 0;
  x.nblk = 1;
  x.tu0 = x.tv0 = 0;
  x.is64 = false;
  x.inside = false;
  if (!x.exists) return x;
  const int U64 = 4 * nt * ntiles;
  if (u < U64) {
    const int m = u / (4 * ntiles), rem = u - m * 4 * ntiles;
    const int part = rem / ntiles, tile = rem - part * ntiles;
    x.col = K + m;
    x.blk = tile * 4 + part;
    x.nblk = 4 * ntiles;
    x.is64 = true;
    const int ty = tile / tilesX, tx = tile - (tile / tilesX) * tilesX;
    x.tu0 = ty * kConvTile + (part >> 1) * (kConvTile / 2);
    x.tv0 = tx * kConvTile + (part & 1) * (kConvTile / 2);
  } else {
    const int v = u - U64;
    const int col = v / ntiles, tile = v - col * ntiles;
    x.col = col;
    x.blk = tile;
    x.nblk = ntiles;
    const int ty = tile / tilesX, tx = tile - (tile / tilesX) * tilesX;
    x.tu0 = ty * kConvTile;
    x.tv0 = tx * kConvTile;
  }
  x.inside = x.tu0 < H && x.tv0 < W;
  return x;
}

// Block barrier ordering LDS only: __syncthreads' release fence also waits
// for every vector-memory operation in flight (loads and stores share one
// counter), which would drain the prefetches that are meant to cross the
// barrier.  Global-memory ordering inside the workgroup is fenced explicitly
// where it is needed.
__device__ __forceinline__ void ws_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Registers of a memory thread's loads, shared by the float and float64
// units (bit patterns in 32-bit words): a block is issued one phase before it
// is used, so it is in flight across a barrier while the compute waves work.
// A thread's staging vectors: slots k < kWsOwnVecs cover the tile's own
// pixels, the rest the halo ring around them.
constexpr int kWsStageVecs = 4;  // 16-byte vectors per thread and stream
constexpr int kWsOwnVecs = 2;
constexpr int kWsEpiVecs = 2;
struct WsStageRaw {
  uint32_t p0[kWsStageVecs][4], r0[kWsStageVecs][4], q0[kWsStageVecs][4], mv[kWsStageVecs][4];
  uint32_t x0[kWsOwnVecs][4];
  uint32_t ix[kWsStageVecs];  // pixel index: a 32-bit offset from each column's base
  bool own[kWsOwnVecs];
};
struct WsEpiRaw {
  uint32_t al[kWsEpiVecs][4];
  uint32_t mv[kWsEpiVecs][4], b0[kWsEpiVecs][4];  // the init and residual modes
  uint32_t ix[kWsEpiVecs];
  bool ok[kWsEpiVecs];
};

// p + ix as a 32-bit byte offset from the (uniform) column base, so the
// load or store takes the base in scalar registers and one vector register
// for the offset (D < 2^28 keeps the offset below 2^31)
template <typename T>
__device__ __forceinline__ T* at(T* base, uint32_t ix) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<C*>(base) + ix * (uint32_t)sizeof(T));
}

__device__ __forceinline__ void raw_load16(uint32_t (&w)[4], const void* p) {
  const uint4 x = *reinterpret_cast<const uint4*>(p);
  w[0] = x.x;
  w[1] = x.y;
  w[2] = x.z;
  w[3] = x.w;
}
__device__ __forceinline__ void raw_load8(uint32_t (&w)[4], const void* p) {
  const uint2 x = *reinterpret_cast<const uint2*>(p);
  w[0] = x.x;
  w[1] = x.y;
}
// element n of a 16-byte vector of T held as words
template <typename T>
__device__ __forceinline__ T raw_get(const uint32_t (&w)[4], int n) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float(w[n]);
  } else {
    return __hiloint2double((int)w[2 * n + 1], (int)w[2 * n]);
  }
}
template <typename T>
__device__ __forceinline__ void vload(T (&v)[16 / sizeof(T)], const T* p) {
  if constexpr (sizeof(T) == 4) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
  } else {
    const double2 x = *reinterpret_cast<const double2*>(p);
    v[0] = x.x;
    v[1] = x.y;
  }
}
template <typename T>
__device__ __forceinline__ void vstore(T* p, const T (&v)[16 / sizeof(T)]) {
  if constexpr (sizeof(T) == 4)
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  else
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
}

// Stores of a unit's own pixels as raw buffer stores: a lane or unit that
// must not store is given an offset (or a record count) outside the buffer,
// which the hardware drops.  So the staging issues the same number of
// stores on every path, and the compiler's count of memory operations in
// flight after the epilogue's alpha loads is exact (a branch around the
// stores would make it wait for them too: loads and stores retire in order).
typedef unsigned int ws_u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kWsNoStore = 0x80000000u;  // beyond every column (D < 2^28)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ws_rsrc(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ void ws_bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, const T (&v)[16 / sizeof(T)]) {
  ws_u32x4 w;
  __builtin_memcpy(&w, v, 16);
  __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)off, 0, 0);
}

// The staged region is [-2c, TILE + 2c)^2 around the tile (ConvGeom: SPH =
// SPW = TILE + 4c for c even), in 16-byte vectors of N values: slot k of
// thread mt holds own vector mt + 512 k (k < KOWN; TILE x TILE/N of them,
// KOWN 512 each), else halo vector h = mt + 512 (k - KOWN): the 2c top rows,
// the 2c bottom rows, then the 2c/N vectors left and right of each tile row.
template <int KS, int TILE, typename T>
struct WsStageMap {
  using G = ConvGeom<KS, TILE>;
  static constexpr int c2 = 2 * G::c, N = 16 / sizeof(T), VW = G::SPW / N, VT = TILE / N, SV = c2 / N;
  static constexpr int NOWN = TILE * VT, KOWN = NOWN / kWsMemory;
  static constexpr int NHALO = G::SPH * VW - NOWN, KHALO = (NHALO + kWsMemory - 1) / kWsMemory;
  static_assert(G::SPW == TILE + 2 * c2 && G::SPH == TILE + 2 * c2, "region is the tile plus 2c");
  static_assert(NOWN % kWsMemory == 0 && KOWN <= kWsOwnVecs && KOWN + KHALO <= kWsStageVecs, "slots");
  // region coordinates (row, column) of slot k of thread mt
  __device__ __forceinline__ static void pos(int mt, int k, int& i, int& j) {
    if (k < KOWN) {
      const int e = mt + k * kWsMemory;
      i = c2 + e / VT;
      j = c2 + (e - (e / VT) * VT) * N;
    } else {
      const int h = mt + (k - KOWN) * kWsMemory, top = c2 * VW;
      if (h < top) {
        i = h / VW;
        j = (h - (h / VW) * VW) * N;
      } else if (h < 2 * top) {
        i = c2 + TILE + (h - top) / VW;
        j = (h - top - ((h - top) / VW) * VW) * N;
      } else {
        const int r = h - 2 * top, q = r % (2 * SV);
        i = c2 + r / (2 * SV);
        j = q < SV ? q * N : c2 + TILE + (q - SV) * N;
      }
    }
  }
  // whether slot k exists for thread mt (only the last halo slot is partial,
  // and it is a whole number of waves)
  __device__ __forceinline__ static bool exists(int mt, int k) {
    return k < KOWN || (k < KOWN + KHALO && mt + (k - KOWN) * kWsMemory < NHALO);
  }
};

// ws_stage_load issues a thread's staging loads of p, r, q (and M^-1) over
// the region, wrapped circularly (H and W are at least one period of the
// region, so a wrap is one compare and add; W a multiple of 4 keeps each
// vector in one period), and x on the own pixels; ws_stage_finish applies
// the previous CG update (r' = r - a q, z = M^-1 r', p' = z + b p,
// x += a p), writes p' to the LDS region, r' and M^-1 of the own pixels to
// sR, sM (TILE x TILE, for the epilogue), x, r', p' of the own pixels inside
// the image to memory, and adds their r'^T z and r'^T r' to rz, rr.
// Slots [K0, K1) of a thread's staging loads (the caller issues the own
// slots and the halo slots at different points of phase 1).
template <int KS, int TILE, typename T, bool PRE, int MD, int K0, int K1>
__device__ __forceinline__ void ws_stage_load(WsStageRaw& g, const T* __restrict__ P0, const T* __restrict__ R0,
                                              const T* __restrict__ Q0, const T* __restrict__ X,
                                              const float* __restrict__ minv, int H, int W, int tu0, int tv0,
                                              int mt) {
  using M = WsStageMap<KS, TILE, T>;
#pragma unroll
  for (int k = K0; k < (K1 < M::KOWN + M::KHALO ? K1 : M::KOWN + M::KHALO); ++k) {
    if (!M::exists(mt, k)) continue;
    int i, j;
    M::pos(mt, k, i, j);
    int u = tu0 - M::c2 + i, v = tv0 - M::c2 + j;
    if (k < M::KOWN) g.own[k] = u < H && v < W;
    u = u < 0 ? u + H : (u >= H ? u - H : u);
    v = v < 0 ? v + W : (v >= W ? v - W : v);
    g.ix[k] = (uint32_t)(u * W + v);
    raw_load16(g.p0[k], at(P0, g.ix[k]));
    // the fused iteration needs r, q, M^-1 over the region and x on the own
    // pixels; the pass r and M^-1 on the own pixels (for its dots).  (k is a
    // constant once the loop is unrolled, so these tests are not branches.)
    const bool rm = MD == kWsFused || (MD == kWsPass && k < M::KOWN);
    if (rm) raw_load16(g.r0[k], at(R0, g.ix[k]));
    if constexpr (MD == kWsFused) raw_load16(g.q0[k], at(Q0, g.ix[k]));
    if constexpr (PRE) {
      if (rm) {
        if constexpr (sizeof(T) == 4)
          raw_load16(g.mv[k], at(minv, g.ix[k]));
        else
          raw_load8(g.mv[k], at(minv, g.ix[k]));
      }
    }
    if constexpr (MD == kWsFused) {
      if (k < M::KOWN) raw_load16(g.x0[k < M::KOWN ? k : 0], at(X, g.ix[k]));
    }
  }
}

// In the pass and apply modes nothing is updated: p' = p (and r' = r on the
// own pixels, for the pass's dots), and nothing is written to memory.
template <int KS, int TILE, typename T, int MD>
__device__ __forceinline__ void ws_stage_finish(const WsStageRaw& g, T* __restrict__ X, T* __restrict__ P1,
                                                T* __restrict__ R1, uint32_t col_bytes, bool precond, bool valid,
                                                T a, T b, int mt, T* sP, T* sR, T* sM, double& rz, double& rr) {
  using M = WsStageMap<KS, TILE, T>;
  constexpr int N = M::N;
  const uint32_t nb = valid ? col_bytes : 0u;
  const __amdgpu_buffer_rsrc_t rX = ws_rsrc(X, nb), rR = ws_rsrc(R1, nb), rP = ws_rsrc(P1, nb);
#pragma unroll
  for (int k = 0; k < M::KOWN + M::KHALO; ++k) {
    if (!M::exists(mt, k)) continue;
    const bool own = valid && k < M::KOWN && g.own[k < M::KOWN ? k : 0];
    T r1[N], p1[N], x1[N], mv[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const T p0 = raw_get<T>(g.p0[k], n);
      if constexpr (MD == kWsFused) {
        r1[n] = fma(-a, raw_get<T>(g.q0[k], n), raw_get<T>(g.r0[k], n));
        mv[n] = precond ? (T)__uint_as_float(g.mv[k][n]) : T(1);
        const T z = precond ? mv[n] * r1[n] : r1[n];
        p1[n] = fma(b, p0, z);
        if (k < M::KOWN) {
          x1[n] = fma(a, p0, raw_get<T>(g.x0[k < M::KOWN ? k : 0], n));
          if (own) {
            rz += (double)r1[n] * (double)z;
            rr += (double)r1[n] * (double)r1[n];
          }
        }
      } else {
        p1[n] = p0;
        if (MD == kWsPass && k < M::KOWN) {
          r1[n] = raw_get<T>(g.r0[k], n);
          mv[n] = precond ? (T)__uint_as_float(g.mv[k][n]) : T(1);
        }
      }
    }
    if constexpr (MD == kWsFused) {
      if (k < M::KOWN) {
        const uint32_t off = own ? g.ix[k] * (uint32_t)sizeof(T) : kWsNoStore;
        ws_bstore<T>(rX, off, x1);
        ws_bstore<T>(rR, off, r1);
        ws_bstore<T>(rP, off, p1);
      }
    }
    if (!valid) continue;
    int i, j;
    M::pos(mt, k, i, j);
    vstore<T>(sP + i * M::G::SPW + j, p1);
    if ((MD == kWsFused || MD == kWsPass) && k < M::KOWN) {
      const int o = (i - M::c2) * TILE + (j - M::c2);
      vstore<T>(sR + o, r1);
      if (precond) vstore<T>(sM + o, mv);
    }
  }
}

// Epilogue of a unit: q = beta Phi^T t + alpha p' on its own pixels (Phi^T t
// in sU, p' in the staged region), written to Q1, and gam = p'^T q,
// del = r'^T M^-1 q, eta = q^T M^-1 q, with r' and M^-1 as the staging left
// them in sR, sM.  ws_epi_load issues the alpha loads (pixels outside the
// image read pixel 0 and are not used), ws_epi_finish does the rest.
template <int TILE, typename T, bool PRE, int MD>
__device__ __forceinline__ void ws_epi_load(WsEpiRaw& g, const float* __restrict__ alpha,
                                            const float* __restrict__ minv, const double* __restrict__ b0, int H,
                                            int W, int tu0, int tv0, int mt) {
  constexpr int N = 16 / sizeof(T), VT = TILE / N, NV = TILE * VT, KE = NV / kWsMemory;
  static_assert(NV % kWsMemory == 0 && KE <= kWsEpiVecs, "epilogue vectors per thread");
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int e = mt + k * kWsMemory;
    const int i = e / VT, j = (e - (e / VT) * VT) * N;
    const int u = tu0 + i, v = tv0 + j;
    g.ok[k] = u < H && v < W;
    g.ix[k] = g.ok[k] ? (uint32_t)(u * W + v) : 0u;
    if constexpr (sizeof(T) == 4)
      raw_load16(g.al[k], at(alpha, g.ix[k]));
    else
      raw_load8(g.al[k], at(alpha, g.ix[k]));
    if constexpr (MD == kWsInit && PRE) {
      if constexpr (sizeof(T) == 4)
        raw_load16(g.mv[k], at(minv, g.ix[k]));
      else
        raw_load8(g.mv[k], at(minv, g.ix[k]));
    }
    // the float64 units' b: the mean column's b0 (a float unit's b is its probe)
    if constexpr ((MD == kWsInit || MD == kWsResid) && sizeof(T) == 8) raw_load16(g.b0[k], at(b0, g.ix[k]));
  }
}

// q of a thread's epilogue vectors, kept in registers until it is stored
// (ws_epi_store, in the next phase: a store issued behind the staging loads
// would wait for them to be accepted)
struct WsEpiOut {
  uint32_t q[kWsEpiVecs][4];  // q (r in the init mode)
  uint32_t z[kWsEpiVecs][4];  // the init mode's z
  uint32_t off[kWsEpiVecs];   // byte offset, or kWsNoStore
};
// The probe signs of 16 / sizeof(T) consecutive pixels from ix (natural
// element order; they share one 64-bit word of the probe's hash): bit
// (j & 63) of SplitMix64 output (t << 48 | k << 32 | j >> 6) + 1.
__device__ __forceinline__ uint64_t ws_probe_word(uint64_t seed, uint32_t t, uint32_t k, uint32_t ix) {
  const uint64_t idx = ((uint64_t)t << 48) | ((uint64_t)k << 32) | (uint64_t)(ix >> 6);
  return splitmix64_mix(seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
}
template <int KS, int TILE, typename T, int MD>
__device__ __forceinline__ void ws_epi_finish(const WsEpiRaw& g, WsEpiOut& out, bool precond, bool valid, T beta,
                                              int mt, const T* sP, const T* sU, const T* sR, const T* sM,
                                              double& gm, double& dl, double& et, uint64_t seed = 0,
                                              uint32_t tt = 0, uint32_t col = 0) {
  using G = ConvGeom<KS, TILE>;
  constexpr int c = G::c, N = 16 / sizeof(T), VT = TILE / N, KE = TILE * VT / kWsMemory;
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const bool use = valid && g.ok[k];
    const int e = mt + k * kWsMemory;
    const int i = e / VT, j = (e - (e / VT) * VT) * N;
    const int o = i * TILE + j;
    T q[N], pv[N], tv[N], rv[N], mv[N];
    vload<T>(pv, sP + (i + 2 * c) * G::SPW + j + 2 * c);
    vload<T>(tv, sU + o);
    if constexpr (MD == kWsFused || MD == kWsPass) {
      vload<T>(rv, sR + o);
      if (precond) vload<T>(mv, sM + o);
    }
    uint64_t w = 0;
    if constexpr ((MD == kWsInit || MD == kWsResid) && sizeof(T) == 4) w = ws_probe_word(seed, tt, col, g.ix[k]);
    T zo[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const T p = pv[n];
      q[n] = fma(beta, tv[n], (T)__uint_as_float(g.al[k][n]) * p);  // as the per-tile kernel
      if constexpr (MD == kWsFused || MD == kWsPass) {
        const double qd = (double)q[n];
        const double mq = precond ? (double)mv[n] * qd : qd;
        if (use) {
          gm += (double)p * qd;
          dl += (double)rv[n] * mq;
          et += qd * mq;
        }
      } else if constexpr (MD == kWsInit || MD == kWsResid) {
        // b: the probe sign (float units), b0 (float64 units); as the
        // start and true-residual kernels form them
        T b;
        if constexpr (sizeof(T) == 4)
          b = ((w >> ((g.ix[k] + n) & 63)) & 1ull) ? -1.0f : 1.0f;
        else
          b = raw_get<T>(g.b0[k], n);
        if constexpr (MD == kWsInit) {
          const T r = b - q[n];
          const T z = precond ? (T)__uint_as_float(g.mv[k][n]) * r : r;
          q[n] = r;
          zo[n] = z;
          if (use) {
            gm += (double)r * (double)z;
            dl += (double)r * (double)r;
            et += sizeof(T) == 4 ? 1.0 : (double)b * (double)b;
          }
        } else {
          const double e = (double)b - (double)q[n];
          if (use) gm += e * e;
        }
      }
    }
    __builtin_memcpy(out.q[k], q, 16);
    if constexpr (MD == kWsInit) __builtin_memcpy(out.z[k], zo, 16);
    out.off[k] = use ? g.ix[k] * (uint32_t)sizeof(T) : kWsNoStore;
  }
}
// q to Q1 (the init mode: r to R1 and z to P1; the residual mode stores
// nothing)
template <int TILE, typename T, int MD>
__device__ __forceinline__ void ws_epi_store(const WsEpiOut& out, T* __restrict__ Q1, T* __restrict__ R1,
                                             T* __restrict__ P1, uint32_t col_bytes, bool valid) {
  constexpr int KE = TILE * (TILE * sizeof(T) / 16) / kWsMemory;
  if constexpr (MD == kWsResid) return;
  const uint32_t nb = valid ? col_bytes : 0u;
  const __amdgpu_buffer_rsrc_t rQ = ws_rsrc(MD == kWsInit ? R1 : Q1, nb), rP = ws_rsrc(P1, nb);
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    ws_u32x4 w;
    __builtin_memcpy(&w, out.q[k], 16);
    __builtin_amdgcn_raw_buffer_store_b128(w, rQ, (int)out.off[k], 0, 0);
    if constexpr (MD == kWsInit) {
      ws_u32x4 wz;
      __builtin_memcpy(&wz, out.z[k], 16);
      __builtin_amdgcn_raw_buffer_store_b128(wz, rP, (int)out.off[k], 0, 0);
    }
  }
}

// A unit's deposit, by compute wave 0 at the end of a phase 2: its five
// sums (wave partials in LDS, summed in wave order) to its row of the
// column's partials.  The columns are summed once, by the launch's last
// workgroup (ws_column_sums): a column completed inside the loop would fall
// to the workgroup that happens to arrive last, which then runs later still
// and is last again for the next column.
__device__ __forceinline__ void ws_deposit(const WsUnit& un, const double* stg, const double* epi,
                                           const ConvReduce& red, int64_t nblk_alloc, int lane) {
  double v = 0.0;
  if (lane < 2) {
    for (int w = 0; w < kWsMemWaves; ++w) v += stg[w * 2 + lane];
  } else if (lane < 5) {
    for (int w = 0; w < kWsMemWaves; ++w) v += epi[w * 3 + lane - 2];
  }
  double* pc = red.parts + (int64_t)un.col * tree_rows(nblk_alloc) * 5;
  if (lane < 5) store_agent(&pc[(int64_t)un.blk * 5 + lane], v);
}

// Whether this workgroup is the launch's last to finish, in two levels: the
// workgroups of each of the 8 XCD groups (blockIdx mod 8) arrive at their
// group's counter, and each group's last arrival at the top counter.  A
// single counter took 256 arrivals on one address, which the memory side
// serialises (~13 us at the end of every launch); here the last workgroup
// waits for at most 32 + 8.  Every store a workgroup made is complete before
// it arrives, and the counters are left at zero.  cnts: 8 counters
// kCounterStride slots apart.
__device__ __forceinline__ bool ws_last_block(uint32_t* cnts, uint32_t* top, int G) {
  __shared__ bool s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    bool last;
    if ((G & 7) == 0) {
      uint32_t* c1 = cnts + (blockIdx.x & 7) * kCounterStride;
      last = __hip_atomic_fetch_add(c1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)(G / 8 - 1);
      if (last) {
        store_agent(c1, 0u);
        last = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 7u;
      }
    } else {
      last = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)(G - 1);
    }
    if (last) store_agent(top, 0u);
    s_last = last;
  }
  __syncthreads();
  return s_last;
}

// The launch's column totals, by its last workgroup: tot[v * nc + col] =
// the sum over the column's rows of value v, in a fixed order.  A column's
// flat array [row * 5 + v] is cut into segments of kWsSeg elements, one per
// wave (two in flight at once): lane l reads the segment at l, l + 64, ...
// (each load one contiguous 512-byte span; these loads are coherent across
// the chip's L2s, so each is a full memory round trip) and adds each element
// to its value's sum in that order; the lanes' sums meet in a fixed
// butterfly, and a column's segments are then added in order.  cp: LDS
// scratch of ws_seg_items(...) * 5 doubles.
constexpr int kWsSegLoads = 20, kWsSeg = 64 * kWsSegLoads;
__host__ __device__ __forceinline__ int ws_col_segs(int n5) { return (n5 + kWsSeg - 1) / kWsSeg; }
__host__ __device__ __forceinline__ int ws_seg_items(int K, int nt, int ntiles) {
  return K * ws_col_segs(5 * ntiles) + nt * ws_col_segs(20 * ntiles);
}
__device__ __forceinline__ void ws_column_sums(const ConvReduce& red, int64_t nblk_alloc, int K, int nt,
                                               int ntiles, double* cp, double* tot) {
  const int nc = K + nt, wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int64_t rows = tree_rows(nblk_alloc);
  const int sF = ws_col_segs(5 * ntiles), sD = ws_col_segs(20 * ntiles), nF = K * sF;
  const int nItems = ws_seg_items(K, nt, ntiles);
  // item -> (column, segment)
  auto where = [&](int i, int& col, int& seg, int& n5) {
    if (i < nF) {
      col = i / sF;
      seg = i - col * sF;
      n5 = 5 * ntiles;
    } else {
      const int j = i - nF;
      col = K + j / sD;
      seg = j - (j / sD) * sD;
      n5 = 20 * ntiles;
    }
  };
  for (int i0 = wave; i0 < nItems; i0 += 2 * nw) {
    double x[2][kWsSegLoads];
    int f0[2], n5[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = i0 + h * nw;
      int col = 0, seg = 0, n = 0;
      if (i < nItems) where(i, col, seg, n);
      const double* pc = red.parts + (int64_t)col * rows * 5;
      f0[h] = seg * kWsSeg;
      n5[h] = i < nItems ? (f0[h] + kWsSeg < n ? f0[h] + kWsSeg : n) : 0;
#pragma unroll
      for (int k = 0; k < kWsSegLoads; ++k) {
        const int f = f0[h] + lane + 64 * k;
        x[h][k] = f < n5[h] ? load_agent(&pc[f]) : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = i0 + h * nw;
      double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < kWsSegLoads; ++k) {
        const int f = f0[h] + lane + 64 * k, r = f - (f / 5) * 5;
#pragma unroll
        for (int v = 0; v < 5; ++v) t[v] += r == v ? x[h][k] : 0.0;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) t[v] = wave_sum(t[v]);
      if (i < nItems && lane < 5)
        cp[i * 5 + lane] = lane == 0 ? t[0] : lane == 1 ? t[1] : lane == 2 ? t[2] : lane == 3 ? t[3] : t[4];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nc * 5; e += blockDim.x) {
    const int col = e / 5, v = e - (e / 5) * 5;
    const int first = col < K ? col * sF : nF + (col - K) * sD, ns = col < K ? sF : sD;
    double t = 0.0;
    for (int g = 0; g < ns; ++g) t += cp[(first + g) * 5 + v];
    tot[v * nc + col] = t;
  }
  __syncthreads();
}

}  // namespace

// The state of one unit kind: float probe columns (column c at c * ldD) or
// float64 mean columns (column K + j at j * ldD).
template <typename T>
struct WsCols {
  const T *P0, *R0, *Q0;
  T *X, *P1, *R1, *Q1;
  const double* B0;  // the mean columns' b0 (the init and residual modes)
  int col0;          // first column of this kind
  int64_t ldD;
  __device__ __forceinline__ int64_t off(int col) const { return (int64_t)(col - col0) * ldD; }
};

struct WsLds {
  unsigned char *sP, *sT, *sU, *sR, *sM;  // 2 staged regions, stage-1 and stage-2 outputs, 2 r', 2 M^-1
  const float* tapsF;
  const double* tapsD;
  const double *a, *b;  // the step scalars a and b of every column
  double (*red_stage)[kWsMemWaves * 2];
  double* red_epi;
};

struct WsGrid {
  int U, ntiles, tilesX, K, nt, H, W, G, slot;
  __device__ __forceinline__ WsUnit unit(int i, int i0, int n) const {
    return ws_unit(i >= 0 && i < n ? (i0 + i) * G + slot : -1, U, ntiles, tilesX, K, nt, H, W);
  }
};

// Steps of a loop over n units of one kind (the workgroup's units i0 ..
// i0 + n - 1): s = -1 .. n, two barriers each.  In step s:
//   phase 1  compute: stage 1 of unit s (sP[s % 2] -> sT)
//            memory:  the staging loads of unit s + 1 issued; the epilogue
//                     of unit s - 1 (sU, sP[(s - 1) % 2], sR and sM
//                     [(s - 1) % 2], the alpha loads issued in the last
//                     phase 2)
//   phase 2  compute: stage 2 of unit s (sT -> sU); wave 0 stores the sums
//                     of unit s - 1
//            memory:  the alpha loads of unit s's epilogue issued; unit
//                     s + 1 staged from the phase-1 loads (the previous CG
//                     update applied, p' written to sP[(s + 1) % 2], r' and
//                     M^-1 to sR and sM [(s + 1) % 2])
// so the staging loads are in flight through stage 1 (the longer stencil
// stage) and the alpha loads through stage 2, and every LDS buffer is
// rewritten only a barrier after its last reader.  The memory waves never
// wait for a store: nothing this launch writes to memory is read back by
// it but the deposits, which the compute wave orders.

// Compute waves: the stencil stages of unit s.
template <int KS, int TILE, typename T, int MD>
__device__ __forceinline__ void ws_compute_loop(const WsGrid& gr, const WsLds& L, const ConvReduce& red,
                                                int64_t nblk_alloc, int i0, int n, int tid) {
  using WG = WsGeom<KS>;
  using G = ConvGeom<KS, TILE>;
  T* const uC = reinterpret_cast<T*>(L.sU);
  T* const sT = reinterpret_cast<T*>(L.sT);
  const bool dep = MD != kWsApply && tid < 64;  // compute wave 0 deposits the units' sums
  for (int s = -1; s <= n; ++s) {
    int ct = tid;  // laundered per step, as in the memory loop
    asm volatile("" : "+v"(ct));
    const WsUnit uc = gr.unit(s, i0, n);
    const bool work = uc.exists && uc.inside;
    const T* const bC = reinterpret_cast<const T*>(L.sP + ((s + 2) & 1) * WG::SP);
    if (work) {
      if constexpr (sizeof(T) == 4 && Stage1W6<KS, TILE>::ok)
        conv_stage1_w6<KS, TILE>(TapsReg<KS>(L.tapsF), bC, sT, ct, kWsCompute);
      else if constexpr (sizeof(T) == 4)
        conv_stage1<KS, TILE, T>(TapsReg<KS>(L.tapsF), bC, sT, ct, kWsCompute);
      else  // float64 quadrants: 4x2 blocks (200 of them) keep all four waves busy
        conv_stage1_blk<KS, TILE, 4, 2, T>(Taps<double>(L.tapsD), bC, sT, ct, kWsCompute);
    }
    ws_barrier();
    if constexpr (sizeof(T) == 4) {
      if (work && ct < G::NB2) {
        T acc[4][4];
        conv_stage2<KS, TILE, T>(TapsReg<KS>(L.tapsF), sT, ct, acc);
        const int bi = ct / (TILE / 4), bj = ct - (ct / (TILE / 4)) * (TILE / 4);
        T* dst = uC + (4 * bi) * TILE + 4 * bj;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T row[4] = {acc[r][0], acc[r][1], acc[r][2], acc[r][3]};
          vstore<T>(dst + r * TILE, *reinterpret_cast<const T(*)[4]>(row));
        }
      }
    } else {  // float64 quadrants: 2x2 blocks, 256 of them, one per compute thread
      using S2 = StageBlk<KS, TILE, 2, 2, T>;
      if (work && ct < S2::NB2) {
        T acc[2][2];
        conv_stage2_blk<KS, TILE, 2, 2, T>(Taps<double>(L.tapsD), sT, ct, acc);
        const int bi = ct / (TILE / 2), bj = ct - (ct / (TILE / 2)) * (TILE / 2);
        T* dst = uC + (2 * bi) * TILE + 2 * bj;
#pragma unroll
        for (int r = 0; r < 2; ++r) vstore<T>(dst + r * TILE, acc[r]);
      }
    }
    // unit s - 1's sums: its staging sums from two steps back, its epilogue
    // sums from this step's phase 1
    const WsUnit ud = gr.unit(s - 1, i0, n);
    if (dep && ud.exists) ws_deposit(ud, L.red_stage[(s + 3) & 3], L.red_epi, red, nblk_alloc, ct);
    ws_barrier();
  }
}

// Memory waves.
template <int KS, int TILE, typename T, bool PRE, int MD>
__device__ __forceinline__ void ws_memory_loop(const WsGrid& gr, const WsLds& L, const WsCols<T>& C,
                                               const float* __restrict__ alpha, const float* __restrict__ minv,
                                               double beta, uint64_t seed, uint32_t tt, int i0, int n, int tid) {
  using WG = WsGeom<KS>;
  constexpr bool precond = PRE;  // a compile-time choice, so every path issues the same loads
  const int mw = (tid - kWsCompute) >> 6, lane = tid & 63;
  const T* const sU = reinterpret_cast<const T*>(L.sU);
  const uint32_t col_bytes = (uint32_t)(gr.H * gr.W) * (uint32_t)sizeof(T);
  WsStageRaw gs;
  WsEpiRaw ge;
  WsEpiOut eo;
  // Every load block and every store is issued on every path, a missing
  // unit's loads from the first tile of the kind's first column (and then not
  // used) and its stores dropped (ws_bstore): the compiler then counts the
  // memory operations in flight exactly, and each consumer waits for its own
  // block only, never for a block or a store issued after it.
  using M = WsStageMap<KS, TILE, T>;
  auto stage_load_own = [&](const WsUnit& u, int mt) {
    const bool v = u.exists && u.inside;
    const int64_t o = v ? C.off(u.col) : 0;
    ws_stage_load<KS, TILE, T, PRE, MD, 0, M::KOWN>(gs, C.P0 + o, C.R0 + o, C.Q0 + o, C.X + o, minv, gr.H, gr.W,
                                                v ? u.tu0 : 0, v ? u.tv0 : 0, mt);
  };
  auto stage_load_halo = [&](const WsUnit& u, int mt) {
    const bool v = u.exists && u.inside;
    const int64_t o = v ? C.off(u.col) : 0;
    ws_stage_load<KS, TILE, T, PRE, MD, M::KOWN, kWsStageVecs>(gs, C.P0 + o, C.R0 + o, C.Q0 + o, C.X + o, minv, gr.H,
                                                           gr.W, v ? u.tu0 : 0, v ? u.tv0 : 0, mt);
  };
  for (int s = -1; s <= n; ++s) {
    // the thread index laundered once per step: the positions derived from
    // it are recomputed each step instead of being hoisted out of the loop
    // (kept live across it they would spill, and a reload from scratch waits
    // for every load in flight)
    int mt = tid - kWsCompute;
    asm volatile("" : "+v"(mt));
    const WsUnit ue = gr.unit(s - 1, i0, n);  // epilogue
    const WsUnit ua = gr.unit(s, i0, n);      // alpha loads for the next epilogue
    const WsUnit un = gr.unit(s + 1, i0, n);  // staged
    const bool ev = ue.exists && ue.inside, av = ua.exists && ua.inside, sv = un.exists && un.inside;
    const int col = sv ? un.col : C.col0;
    // ---------------- phase 1
    // the staging loads of the own pixels first, then the epilogue (it
    // waits only for its alpha block, issued before them), then those of
    // the halo: the loads are in flight through most of stage 1, and the
    // epilogue's work fills the time their issue would stall
    stage_load_own(un, mt);
    {
      double gm = 0.0, dl = 0.0, et = 0.0;
      const int b = (s + 1) & 1;
      ws_epi_finish<KS, TILE, T, MD>(ge, eo, precond, ev, (T)beta, mt,
                                 reinterpret_cast<const T*>(L.sP + b * WG::SP), sU,
                                 reinterpret_cast<const T*>(L.sR + b * WG::SU),
                                 reinterpret_cast<const T*>(L.sM + b * WG::SU), gm, dl, et, seed, tt,
                                 (uint32_t)(ev ? ue.col : 0));
      stage_load_halo(un, mt);
      if (ue.exists) {
        gm = wave_sum(gm);
        dl = wave_sum(dl);
        et = wave_sum(et);
        if (lane == 0) {
          L.red_epi[mw * 3 + 0] = gm;
          L.red_epi[mw * 3 + 1] = dl;
          L.red_epi[mw * 3 + 2] = et;
        }
      }
    }
    ws_barrier();  // the staging loads stay in flight across it
    // ---------------- phase 2
    ws_epi_load<TILE, T, PRE, MD>(ge, alpha, minv, C.B0 + (av ? C.off(ua.col) : 0), gr.H, gr.W, av ? ua.tu0 : 0,
                                  av ? ua.tv0 : 0, mt);
    {
      const int64_t o = ev ? C.off(ue.col) : 0;
      ws_epi_store<TILE, T, MD>(eo, C.Q1 + o, C.R1 + o, C.P1 + o, col_bytes, ev);
    }
    {
      double rz = 0.0, rr = 0.0;
      const int64_t o = sv ? C.off(un.col) : 0;
      const int b = (s + 1) & 1;
      ws_stage_finish<KS, TILE, T, MD>(gs, C.X + o, C.P1 + o, C.R1 + o, col_bytes, precond, sv, (T)L.a[col], (T)L.b[col], mt,
                                   reinterpret_cast<T*>(L.sP + b * WG::SP), reinterpret_cast<T*>(L.sR + b * WG::SU),
                                   reinterpret_cast<T*>(L.sM + b * WG::SU), rz, rr);
      if (un.exists) {
        rz = wave_sum(rz);
        rr = wave_sum(rr);
        if (lane == 0) {
          L.red_stage[(s + 5) & 3][mw * 2 + 0] = rz;
          L.red_stage[(s + 5) & 3][mw * 2 + 1] = rr;
        }
      }
    }
    ws_barrier();  // the alpha loads stay in flight across it
  }
}

template <int KS, bool PRE, int MD>
__global__ __launch_bounds__(kWsThreads) void k_conv_ws(
    const float* __restrict__ taps, int H, int W, int64_t ldD, int K, int nt, int tilesX, int ntiles,
    const float* __restrict__ P0, const float* __restrict__ R0, const float* __restrict__ Q0, float* __restrict__ X,
    float* __restrict__ P1, float* __restrict__ R1, float* __restrict__ Q1, const double* __restrict__ pm0,
    const double* __restrict__ rm0, const double* __restrict__ qm0, double* __restrict__ xm,
    double* __restrict__ pm1, double* __restrict__ rm1, double* __restrict__ qm1, const float* __restrict__ alpha,
    double beta, const float* __restrict__ minv, ConvReduce red, int64_t nblk_alloc, CgScalars* __restrict__ st,
    const double* __restrict__ b0, uint64_t seed, int tt, int only_if_stopped) {
  // a CG iteration does nothing once the solve has stopped; the other modes
  // run at a solve's start or after it.  A residual launch enqueued before the
  // host knows whether the solve has stopped (`only_if_stopped`) does nothing
  // unless it has.
  if ((MD == kWsFused || MD == kWsPass) && st->stop) return;
  if (MD == kWsResid && only_if_stopped && !st->stop) return;
  const CgCtl ctl = load_cg_ctl(st);
  using WG = WsGeom<KS>;
  using GF = typename WG::GF;
  using GD = typename WG::GD;
  __shared__ __align__(16) unsigned char smem[WG::BYTES];
  __shared__ double sTapsD[KS * KS];
  __shared__ float sTapsF[KS * KS];
  __shared__ double red_stage[4][kWsMemWaves * 2];
  __shared__ double red_epi[kWsMemWaves * 3];
  // the step scalars are read once: they do not change until the launch's
  // last workgroup finishes (and a scalar load in the loop would share its
  // wait counter with the LDS reads, at memory latency)
  __shared__ double sA[kMaxCols], sB[kMaxCols];
  const int tid = threadIdx.x;
  if (tid < KS * KS) {
    sTapsD[tid] = (double)taps[tid];
    sTapsF[tid] = taps[tid];
  }
  if (tid < K + nt) {
    sA[tid] = st->a[tid];
    sB[tid] = st->b[tid];
  }
  __syncthreads();
  unsigned char* const sPb = smem;
  unsigned char* const sTb = smem + 2 * WG::SP;
  unsigned char* const sUb = sTb + WG::ST;
  unsigned char* const sRb = sUb + WG::SU;
  unsigned char* const sMb = sRb + 2 * WG::SU;
  const bool isC = tid < kWsCompute;
  const int G = (int)gridDim.x;
  const int wgi = (int)blockIdx.x;
  const int slot = (G & 7) == 0 ? (wgi & 7) * (G >> 3) + (wgi >> 3) : wgi;
  const int U = (4 * nt + K) * ntiles;
  const int N = slot < U ? (U - 1 - slot) / G + 1 : 0;
  // Each role runs its own loops (a barrier counts waves, not code
  // positions): first over the workgroup's float64 units, then over its
  // float units (each loop's registers allocated for one element type), with
  // the schedule described at ws_compute_loop.
  const int U64 = 4 * nt * ntiles;
  const int N64 = slot < U64 ? (U64 - 1 - slot) / G + 1 : 0;
  const int NF = N - N64;
  const WsGrid gr{U, ntiles, tilesX, K, nt, H, W, G, slot};
  const WsLds L{sPb, sTb, sUb, sRb, sMb, sTapsF, sTapsD, sA, sB, red_stage, red_epi};
  if (isC) {
    ws_compute_loop<KS, kConvTile / 2, double, MD>(gr, L, red, nblk_alloc, 0, N64, tid);
    ws_compute_loop<KS, kConvTile, float, MD>(gr, L, red, nblk_alloc, N64, NF, tid);
  } else {
    const WsCols<double> cd{pm0, rm0, qm0, xm, pm1, rm1, qm1, b0, K, ldD};
    const WsCols<float> cf{P0, R0, Q0, X, P1, R1, Q1, nullptr, 0, ldD};
    ws_memory_loop<KS, kConvTile / 2, double, PRE, MD>(gr, L, cd, alpha, minv, beta, seed, (uint32_t)tt, 0, N64, tid);
    ws_memory_loop<KS, kConvTile, float, PRE, MD>(gr, L, cf, alpha, minv, beta, seed, (uint32_t)tt, N64, NF, tid);
  }
  if constexpr (MD != kWsApply) {
    // the last workgroup to finish sums the columns and takes the step's
    // scalars from the totals (gam, del, eta are values 2-4 of a unit's sums)
    __shared__ double tot[5 * kMaxCols];
    if (!ws_last_block(red.cnts, red.cnt_cols, G)) return;
    ws_column_sums(red, nblk_alloc, K, nt, ntiles, reinterpret_cast<double*>(smem), tot);
    if constexpr (MD == kWsFused)
      finish_fused(st, tot, K + nt, ctl);
    else if constexpr (MD == kWsPass)
      finish_step(st, tot + 2 * (K + nt), ctl);
    else if constexpr (MD == kWsInit)
      finish_init_pcg(st, tot + 2 * (K + nt), K + nt);
    else
      finish_true_resid(st, tot + 2 * (K + nt));
  }
}

bool conv_ws_ok(const ConvDims& cd) {
  // kernel sides 1, 5, 9: the staged region then starts on a multiple of
  // four columns (2c = ks - 1), and with W a multiple of four every 16-byte
  // vector of it is aligned
  if (cd.fp64 || cd.perm != 0 || (cd.ks != 1 && cd.ks != 5 && cd.ks != 9) || cd.W % 4 != 0) return false;
  if (cd.K + cd.nt > kMaxCols) return false;
  if ((4 * (int64_t)cd.nt + cd.K) * cd.tilesX * cd.tilesY >= ((int64_t)1 << 30)) return false;
  if (cd.D >= ((int64_t)1 << 28)) return false;  // 32-bit pixel offsets within a column
  // the two-level finish ticket takes 8 of the reduction's counters
  if (tree_counters(conv_pass_blocks(cd)) * (cd.K + cd.nt) < 8) return false;
  // the final column sums' segment partials fit in the LDS staging buffers
  if ((size_t)ws_seg_items(cd.K, cd.nt, cd.tilesX * cd.tilesY) * 5 * sizeof(double) > WsGeom<9>::BYTES / 2)
    return false;
  // the staged regions of both unit kinds wrap at most one period
  const int c = (cd.ks - 1) / 2;
  const int trf = ((kConvTile + 2 * c + 3) / 4) * 4, trd = ((kConvTile / 2 + 2 * c + 3) / 4) * 4;
  const int xw = ((cd.ks + 3 + 3) / 4) * 4;
  const int need_h = trf > trd ? trf : trd;
  const int need_w = (trf + xw - 4 - 2 * c) > (trd + xw - 4 - 2 * c) ? (trf + xw - 4 - 2 * c) : (trd + xw - 4 - 2 * c);
  return cd.H >= need_h && cd.W >= need_w;
}

template <int MD>
static hipError_t ws_launch(const ConvDims& cd, int grid, const float* taps, const void* P0, const void* R0,
                            const void* Q0, void* X, void* P1, void* R1, void* Q1, const double* pm0,
                            const double* rm0, const double* qm0, double* xm, double* pm1, double* rm1, double* qm1,
                            const float* alpha, double beta, const float* minv, const ConvReduce& red, CgScalars* st,
                            hipStream_t s, const double* b0 = nullptr, uint64_t seed = 0, int t = 0,
                            int only_if_stopped = 0) {
  if (!conv_ws_ok(cd) || grid < 1) return hipErrorInvalidValue;
  const int ntiles = cd.tilesX * cd.tilesY;
  const int64_t nblk_alloc = conv_pass_blocks(cd);
#define COFEM_WS_LAUNCH(KS, PRE)                                                                                   \
  hipLaunchKernelGGL((k_conv_ws<KS, PRE, MD>), dim3((unsigned)grid), dim3(kWsThreads), 0, s, taps, cd.H, cd.W,     \
                     cd.ldD, cd.K, cd.nt, cd.tilesX, ntiles, static_cast<const float*>(P0),                        \
                     static_cast<const float*>(R0), static_cast<const float*>(Q0), static_cast<float*>(X),         \
                     static_cast<float*>(P1), static_cast<float*>(R1), static_cast<float*>(Q1), pm0, rm0, qm0, xm, \
                     pm1, rm1, qm1, alpha, beta, minv, red, nblk_alloc, st, b0, seed, t, only_if_stopped)
#define COFEM_WS_CASE(KS)                       \
  case KS:                                      \
    if constexpr (MD == kWsApply || MD == kWsResid) \
      COFEM_WS_LAUNCH(KS, false); /* no M^-1 */ \
    else if (minv)                              \
      COFEM_WS_LAUNCH(KS, true);                \
    else                                        \
      COFEM_WS_LAUNCH(KS, false);               \
    break;
  switch (cd.ks) {
    COFEM_WS_CASE(1)
    COFEM_WS_CASE(5)
    COFEM_WS_CASE(9)
    default:
      return hipErrorInvalidValue;
  }
#undef COFEM_WS_CASE
#undef COFEM_WS_LAUNCH
  return hipGetLastError();
}

hipError_t conv_fused_ws(const ConvDims& cd, int grid, const float* taps, const ConvState& s0, const ConvState& s1,
                         void* X, double* xm, const float* alpha, double beta, const float* minv,
                         const ConvReduce& red, CgScalars* st, hipStream_t s) {
  return ws_launch<kWsFused>(cd, grid, taps, s0.P, s0.R, s0.Q, X, s1.P, s1.R, s1.Q, s0.pm, s0.rm, s0.qm, xm, s1.pm,
                             s1.rm, s1.qm, alpha, beta, minv, red, st, s);
}

hipError_t conv_pass_ws(const ConvDims& cd, int grid, const float* taps, const void* P, const double* pm,
                        const void* R, const double* rm, const float* alpha, double beta, void* Q, double* qm,
                        const ConvReduce& red, CgScalars* st, int apply_only, hipStream_t s, const float* minv) {
  if (apply_only)
    return ws_launch<kWsApply>(cd, grid, taps, P, nullptr, nullptr, nullptr, nullptr, nullptr, Q, pm, nullptr,
                               nullptr, nullptr, nullptr, nullptr, qm, alpha, beta, nullptr, red, st, s);
  return ws_launch<kWsPass>(cd, grid, taps, P, R, nullptr, nullptr, nullptr, nullptr, Q, pm, rm, nullptr, nullptr,
                            nullptr, nullptr, qm, alpha, beta, minv, red, st, s);
}

hipError_t conv_init_ws(const ConvDims& cd, int grid, const float* taps, uint64_t seed, int t, const double* b0,
                        const float* minv, const void* X, const double* xm, void* R, void* P, double* rm,
                        double* pm, const float* alpha, double beta, const ConvReduce& red, CgScalars* st,
                        hipStream_t s) {
  if (cd.perm != 0) return hipErrorInvalidValue;  // the probe words assume the natural order
  return ws_launch<kWsInit>(cd, grid, taps, X, nullptr, nullptr, nullptr, P, R, nullptr, xm, nullptr, nullptr,
                            nullptr, pm, rm, nullptr, alpha, beta, minv, red, st, s, b0, seed, t);
}

hipError_t conv_resid_ws(const ConvDims& cd, int grid, const float* taps, uint64_t seed, int t, const double* b0,
                         const void* X, const double* xm, const float* alpha, double beta, const ConvReduce& red,
                         CgScalars* st, hipStream_t s, bool only_if_stopped) {
  if (cd.perm != 0) return hipErrorInvalidValue;
  return ws_launch<kWsResid>(cd, grid, taps, X, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, xm, nullptr,
                             nullptr, nullptr, nullptr, nullptr, nullptr, alpha, beta, nullptr, red, st, s, b0, seed,
                             t, only_if_stopped ? 1 : 0);
}

}  // namespace cofem
