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
//   compute waves (4): stage 1 and stage 2 of unit n (LDS only);
//   memory waves (8):  staging of unit n + 1 and the epilogue of unit n - 1.
// Step s of a workgroup's loop has two phases separated by block barriers:
//   phase 1: compute: stage 1 of unit s-1 (sP[(s-1)%3] -> sT)
//            memory:  epilogue of unit s-2 (sU[s%2], sP[(s-2)%3]), staging of
//                     unit s, first part (-> sP[s%3])
//   phase 2: compute: stage 2 of unit s-1 (sT -> sU[(s-1)%2])
//            memory:  staging of unit s, second part; the partial sums of
//                     unit s-2 deposited and, for a column's last unit, the
//                     column summed
// so sP is triple-buffered (staged at s, read at s+1 and s+2) and sU
// double-buffered.  Every wave runs the same number of steps and exactly two
// barriers per step; the role functions contain none.
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
  static constexpr size_t SU = mx(kConvTile * kConvTile * 4, (kConvTile / 2) * (kConvTile / 2) * 8);
  static constexpr size_t BYTES = 3 * SP + ST + 2 * SU;
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
  uint32_t al[kWsEpiVecs][4], mv[kWsEpiVecs][4], r0[kWsEpiVecs][4], q0[kWsEpiVecs][4];
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
__device__ __forceinline__ void vstore(T* p, const T (&v)[16 / sizeof(T)]) {
  if constexpr (sizeof(T) == 4)
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  else
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
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
// x += a p), writes p' to LDS and x, r', p' of the own pixels inside the
// image to memory, and adds their r'^T z and r'^T r' to rz, rr.
template <int KS, int TILE, typename T>
__device__ __forceinline__ void ws_stage_load(WsStageRaw& g, const T* __restrict__ P0, const T* __restrict__ R0,
                                              const T* __restrict__ Q0, const T* __restrict__ X,
                                              const float* __restrict__ minv, int H, int W, int tu0, int tv0,
                                              int mt) {
  using M = WsStageMap<KS, TILE, T>;
#pragma unroll
  for (int k = 0; k < M::KOWN + M::KHALO; ++k) {
    if (!M::exists(mt, k)) continue;
    int i, j;
    M::pos(mt, k, i, j);
    int u = tu0 - M::c2 + i, v = tv0 - M::c2 + j;
    if (k < M::KOWN) g.own[k] = u < H && v < W;
    u = u < 0 ? u + H : (u >= H ? u - H : u);
    v = v < 0 ? v + W : (v >= W ? v - W : v);
    g.ix[k] = (uint32_t)(u * W + v);
    raw_load16(g.p0[k], at(P0, g.ix[k]));
    raw_load16(g.r0[k], at(R0, g.ix[k]));
    raw_load16(g.q0[k], at(Q0, g.ix[k]));
    if (minv) {
      if constexpr (sizeof(T) == 4)
        raw_load16(g.mv[k], at(minv, g.ix[k]));
      else
        raw_load8(g.mv[k], at(minv, g.ix[k]));
    }
    if (k < M::KOWN) raw_load16(g.x0[k < M::KOWN ? k : 0], at(X, g.ix[k]));
  }
}

template <int KS, int TILE, typename T>
__device__ __forceinline__ void ws_stage_finish(const WsStageRaw& g, T* __restrict__ X, T* __restrict__ P1,
                                                T* __restrict__ R1, bool precond, T a, T b, int mt, T* sP,
                                                double& rz, double& rr) {
  using M = WsStageMap<KS, TILE, T>;
  constexpr int N = M::N;
#pragma unroll
  for (int k = 0; k < M::KOWN + M::KHALO; ++k) {
    if (!M::exists(mt, k)) continue;
    const bool own = k < M::KOWN && g.own[k < M::KOWN ? k : 0];
    T r1[N], p1[N], x1[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const T p0 = raw_get<T>(g.p0[k], n);
      r1[n] = fma(-a, raw_get<T>(g.q0[k], n), raw_get<T>(g.r0[k], n));
      const T z = precond ? (T)__uint_as_float(g.mv[k][n]) * r1[n] : r1[n];
      p1[n] = fma(b, p0, z);
      if (k < M::KOWN) {
        x1[n] = fma(a, p0, raw_get<T>(g.x0[k < M::KOWN ? k : 0], n));
        if (own) {
          rz += (double)r1[n] * (double)z;
          rr += (double)r1[n] * (double)r1[n];
        }
      }
    }
    int i, j;
    M::pos(mt, k, i, j);
    vstore<T>(sP + i * M::G::SPW + j, p1);
    if (own) {
      vstore<T>(at(X, g.ix[k]), x1);
      vstore<T>(at(R1, g.ix[k]), r1);
      vstore<T>(at(P1, g.ix[k]), p1);
    }
  }
}

// Epilogue of a unit: q = beta Phi^T t + alpha p' on its own pixels (Phi^T t
// in sU, p' in the staged region), written to Q1, and gam = p'^T q,
// del = r'^T M^-1 q, eta = q^T M^-1 q, with r' = r - a q recomputed from the
// previous iteration's r and q (as the staging formed it; those buffers are
// not written in this launch, so no ordering against the staging's stores
// is needed).  Loads (alpha, M^-1, r, q) by ws_epi_load (pixels outside the
// image read pixel 0 and are not used), the rest by ws_epi_finish.
template <int TILE, typename T>
__device__ __forceinline__ void ws_epi_load(WsEpiRaw& g, const T* __restrict__ R0, const T* __restrict__ Q0,
                                            const float* __restrict__ alpha, const float* __restrict__ minv, int H,
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
    raw_load16(g.r0[k], at(R0, g.ix[k]));
    raw_load16(g.q0[k], at(Q0, g.ix[k]));
    if constexpr (sizeof(T) == 4) {
      raw_load16(g.al[k], at(alpha, g.ix[k]));
      if (minv) raw_load16(g.mv[k], at(minv, g.ix[k]));
    } else {
      raw_load8(g.al[k], at(alpha, g.ix[k]));
      if (minv) raw_load8(g.mv[k], at(minv, g.ix[k]));
    }
  }
}

template <int KS, int TILE, typename T>
__device__ __forceinline__ void ws_epi_finish(const WsEpiRaw& g, T* __restrict__ Q1, bool precond, T a, T beta,
                                              int mt, const T* sP, const T* sU, double& gm, double& dl, double& et) {
  using G = ConvGeom<KS, TILE>;
  constexpr int c = G::c, N = 16 / sizeof(T), VT = TILE / N, KE = TILE * VT / kWsMemory;
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    if (!g.ok[k]) continue;
    const int e = mt + k * kWsMemory;
    const int i = e / VT, j = (e - (e / VT) * VT) * N;
    const T* ps = sP + (i + 2 * c) * G::SPW + j + 2 * c;
    const T* ts = sU + i * TILE + j;
    T q[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const T p = ps[n];
      q[n] = fma(beta, ts[n], (T)__uint_as_float(g.al[k][n]) * p);  // as the per-tile kernel
      const T r1 = fma(-a, raw_get<T>(g.q0[k], n), raw_get<T>(g.r0[k], n));
      const double qd = (double)q[n];
      const double mq = precond ? (double)__uint_as_float(g.mv[k][n]) * qd : qd;
      gm += (double)p * qd;
      dl += (double)r1 * mq;
      et += qd * mq;
    }
    vstore<T>(at(Q1, g.ix[k]), q);
  }
}

// One wave (all 64 lanes): the unit's five sums (wave partials in LDS, summed
// in wave order) to the column's partial rows; the deposit that completes the
// column sums its rows (lane l: rows l, l + 64, ... in order, then a fixed
// butterfly) into colsum and re-arms the column's counter.
__device__ __forceinline__ void ws_deposit(const WsUnit& un, const double* stg, const double* epi,
                                           const ConvReduce& red, int64_t nblk_alloc, int lane) {
  double v = 0.0;
  if (lane < 2) {
    for (int w = 0; w < kWsMemWaves; ++w) v += stg[w * 2 + lane];
  } else if (lane < 5) {
    for (int w = 0; w < kWsMemWaves; ++w) v += epi[w * 3 + lane - 2];
  }
  double* pc = red.parts + (int64_t)un.col * tree_rows(nblk_alloc) * 5;
  uint32_t* cnt = red.cnts + (int64_t)un.col * tree_counters(nblk_alloc) * kCounterStride;
  if (lane < 5) store_agent(&pc[(int64_t)un.blk * 5 + lane], v);
  __builtin_amdgcn_s_waitcnt(0);
  uint32_t prev = 0;
  if (lane == 0) prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  prev = __shfl(prev, 0, 64);
  if (prev != (uint32_t)(un.nblk - 1)) return;
  const int n5 = un.nblk * 5;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0;
  constexpr int CH = 8;
  for (int f0 = 0; f0 < n5; f0 += 64 * CH) {
    double x[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int f = f0 + lane + 64 * k;
      x[k] = f < n5 ? load_agent(&pc[f]) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int f = f0 + lane + 64 * k;
      const int r = f - (f / 5) * 5;
      t0 += r == 0 ? x[k] : 0.0;
      t1 += r == 1 ? x[k] : 0.0;
      t2 += r == 2 ? x[k] : 0.0;
      t3 += r == 3 ? x[k] : 0.0;
      t4 += r == 4 ? x[k] : 0.0;
    }
  }
  t0 = wave_sum(t0);
  t1 = wave_sum(t1);
  t2 = wave_sum(t2);
  t3 = wave_sum(t3);
  t4 = wave_sum(t4);
  const double mine = lane == 0 ? t0 : lane == 1 ? t1 : lane == 2 ? t2 : lane == 3 ? t3 : t4;
  if (lane < 5) store_agent(&red.colsum[un.col * 5 + lane], mine);
  if (lane == 0) store_agent(cnt, 0u);
}

}  // namespace

// The state of one unit kind: float probe columns (column c at c * ldD) or
// float64 mean columns (column K + j at j * ldD).
template <typename T>
struct WsCols {
  const T *P0, *R0, *Q0;
  T *X, *P1, *R1, *Q1;
  int col0;  // first column of this kind
  int64_t ldD;
  __device__ __forceinline__ int64_t off(int col) const { return (int64_t)(col - col0) * ldD; }
};

struct WsLds {
  unsigned char *sP, *sT, *sU;  // 3 staged regions, stage-1 output, 2 stage-2 outputs
  const float* tapsF;
  const double* tapsD;
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
// i0 + n - 1): s = -1 .. n + 1, two barriers each.  In step s:
//   phase 1  compute: stage 1 of unit s (sP[s % 3] -> sT)
//            memory:  the loads of unit s + 1's staging and unit s - 1's
//                     epilogue issued
//   phase 2  compute: stage 2 of unit s (sT -> sU[s % 2])
//            memory:  unit s - 2's sums deposited (wave 0), unit s + 1 staged
//                     (the previous CG update applied, p' written to
//                     sP[(s + 1) % 3]) and unit s - 1's epilogue
//                     (sP[(s - 1) % 3], sU[(s - 1) % 2]), from those loads
// So both load blocks are in flight across a barrier while the compute waves
// run stage 1.  Nothing this launch writes is read back by it, so no wait for
// stores is needed but the deposit's own.

// Compute waves: the stencil stages of unit s.
template <int KS, int TILE, typename T>
__device__ __forceinline__ void ws_compute_loop(const WsGrid& gr, const WsLds& L, int i0, int n, int tid) {
  using WG = WsGeom<KS>;
  using G = ConvGeom<KS, TILE>;
  for (int s = -1; s <= n + 1; ++s) {
    int ct = tid;  // laundered per step, as in the memory loop
    asm volatile("" : "+v"(ct));
    const WsUnit uc = gr.unit(s, i0, n);
    const bool work = uc.exists && uc.inside;
    const T* const bC = reinterpret_cast<const T*>(L.sP + ((s + 3) % 3) * WG::SP);
    T* const uC = reinterpret_cast<T*>(L.sU + ((s + 2) & 1) * WG::SU);
    T* const sT = reinterpret_cast<T*>(L.sT);
    if (work) {
      if constexpr (sizeof(T) == 4 && Stage1W6<KS, TILE>::ok)
        conv_stage1_w6<KS, TILE>(TapsReg<KS>(L.tapsF), bC, sT, ct, kWsCompute);
      else if constexpr (sizeof(T) == 4)
        conv_stage1<KS, TILE, T>(TapsReg<KS>(L.tapsF), bC, sT, ct, kWsCompute);
      else
        conv_stage1<KS, TILE, T>(Taps<double>(L.tapsD), bC, sT, ct, kWsCompute);
    }
    ws_barrier();
    if (work && ct < G::NB2) {
      T acc[4][4];
      if constexpr (sizeof(T) == 4)
        conv_stage2<KS, TILE, T>(TapsReg<KS>(L.tapsF), sT, ct, acc);
      else
        conv_stage2<KS, TILE, T>(Taps<double>(L.tapsD), sT, ct, acc);
      const int bi = ct / (TILE / 4), bj = ct - (ct / (TILE / 4)) * (TILE / 4);
      T* dst = uC + (4 * bi) * TILE + 4 * bj;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T row[4] = {acc[r][0], acc[r][1], acc[r][2], acc[r][3]};
        vstore<T>(dst + r * TILE, *reinterpret_cast<const T(*)[16 / sizeof(T)]>(row));
        if constexpr (sizeof(T) == 8)
          vstore<T>(dst + r * TILE + 2, *reinterpret_cast<const T(*)[2]>(row + 2));
      }
    }
    ws_barrier();
  }
}

// Memory waves.
template <int KS, int TILE, typename T>
__device__ __forceinline__ void ws_memory_loop(const WsGrid& gr, const WsLds& L, const WsCols<T>& C,
                                               const float* __restrict__ alpha, const float* __restrict__ minv,
                                               double beta, const CgScalars* st, const ConvReduce& red,
                                               int64_t nblk_alloc, int i0, int n, int tid) {
  using WG = WsGeom<KS>;
  const bool precond = minv != nullptr;
  const int mw = (tid - kWsCompute) >> 6, lane = tid & 63;
  WsStageRaw gs;
  WsEpiRaw ge;
  for (int s = -1; s <= n + 1; ++s) {
    // the thread index laundered once per step: the positions derived from
    // it are recomputed each step instead of being hoisted out of the loop
    // (kept live across it they would spill, and a reload from scratch waits
    // for every load in flight)
    int mt = tid - kWsCompute;
    asm volatile("" : "+v"(mt));
    const WsUnit un = gr.unit(s + 1, i0, n);  // staged
    const WsUnit ue = gr.unit(s - 1, i0, n);  // epilogue
    const WsUnit ud = gr.unit(s - 2, i0, n);  // deposited
    // ---------------- phase 1
    if (un.exists && un.inside) {
      const int64_t o = C.off(un.col);
      ws_stage_load<KS, TILE, T>(gs, C.P0 + o, C.R0 + o, C.Q0 + o, C.X + o, minv, gr.H, gr.W, un.tu0, un.tv0, mt);
    }
    if (ue.exists && ue.inside) {
      const int64_t o = C.off(ue.col);
      ws_epi_load<TILE, T>(ge, C.R0 + o, C.Q0 + o, alpha, minv, gr.H, gr.W, ue.tu0, ue.tv0, mt);
    }
    ws_barrier();  // the loads just issued stay in flight across it
    // ---------------- phase 2
    // wave 0 deposits unit s - 2 first: its wait for the deposit's stores then
    // covers only the loads this phase consumes anyway
    if (mw == 0 && ud.exists)
      ws_deposit(ud, L.red_stage[(s + 2) & 3], L.red_epi + (s & 1) * kWsMemWaves * 3, red, nblk_alloc, lane);
    if (un.exists) {
      double rz = 0.0, rr = 0.0;
      if (un.inside) {
        const int64_t o = C.off(un.col);
        ws_stage_finish<KS, TILE, T>(gs, C.X + o, C.P1 + o, C.R1 + o, precond, (T)st->a[un.col], (T)st->b[un.col],
                                     mt, reinterpret_cast<T*>(L.sP + ((s + 4) % 3) * WG::SP), rz, rr);
      }
      rz = wave_sum(rz);
      rr = wave_sum(rr);
      if (lane == 0) {
        L.red_stage[(s + 5) & 3][mw * 2 + 0] = rz;
        L.red_stage[(s + 5) & 3][mw * 2 + 1] = rr;
      }
    }
    if (ue.exists) {
      double gm = 0.0, dl = 0.0, et = 0.0;
      if (ue.inside) {
        const int64_t o = C.off(ue.col);
        ws_epi_finish<KS, TILE, T>(ge, C.Q1 + o, precond, (T)st->a[ue.col], (T)beta, mt,
                                   reinterpret_cast<const T*>(L.sP + ((s + 2) % 3) * WG::SP),
                                   reinterpret_cast<const T*>(L.sU + ((s + 1) & 1) * WG::SU), gm, dl, et);
      }
      gm = wave_sum(gm);
      dl = wave_sum(dl);
      et = wave_sum(et);
      if (lane == 0) {
        double* re = L.red_epi + ((s + 1) & 1) * kWsMemWaves * 3;
        re[mw * 3 + 0] = gm;
        re[mw * 3 + 1] = dl;
        re[mw * 3 + 2] = et;
      }
    }
    ws_barrier();
  }
}

template <int KS>
__global__ __launch_bounds__(kWsThreads) void k_conv_ws(
    const float* __restrict__ taps, int H, int W, int64_t ldD, int K, int nt, int tilesX, int ntiles,
    const float* __restrict__ P0, const float* __restrict__ R0, const float* __restrict__ Q0, float* __restrict__ X,
    float* __restrict__ P1, float* __restrict__ R1, float* __restrict__ Q1, const double* __restrict__ pm0,
    const double* __restrict__ rm0, const double* __restrict__ qm0, double* __restrict__ xm,
    double* __restrict__ pm1, double* __restrict__ rm1, double* __restrict__ qm1, const float* __restrict__ alpha,
    double beta, const float* __restrict__ minv, ConvReduce red, int64_t nblk_alloc, CgScalars* __restrict__ st) {
  if (st->stop) return;
  const CgCtl ctl = load_cg_ctl(st);
  using WG = WsGeom<KS>;
  using GF = typename WG::GF;
  using GD = typename WG::GD;
  __shared__ __align__(16) unsigned char smem[WG::BYTES];
  __shared__ double sTapsD[KS * KS];
  __shared__ float sTapsF[KS * KS];
  __shared__ double red_stage[4][kWsMemWaves * 2];
  __shared__ double red_epi[2 * kWsMemWaves * 3];
  const int tid = threadIdx.x;
  if (tid < KS * KS) {
    sTapsD[tid] = (double)taps[tid];
    sTapsF[tid] = taps[tid];
  }
  __syncthreads();
  unsigned char* const sPb = smem;
  unsigned char* const sTb = smem + 3 * WG::SP;
  unsigned char* const sUb = sTb + WG::ST;
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
  const WsLds L{sPb, sTb, sUb, sTapsF, sTapsD, red_stage, red_epi};
  if (isC) {
    ws_compute_loop<KS, kConvTile / 2, double>(gr, L, 0, N64, tid);
    ws_compute_loop<KS, kConvTile, float>(gr, L, N64, NF, tid);
  } else {
    const WsCols<double> cd{pm0, rm0, qm0, xm, pm1, rm1, qm1, K, ldD};
    const WsCols<float> cf{P0, R0, Q0, X, P1, R1, Q1, 0, ldD};
    ws_memory_loop<KS, kConvTile / 2, double>(gr, L, cd, alpha, minv, beta, st, red, nblk_alloc, 0, N64, tid);
    ws_memory_loop<KS, kConvTile, float>(gr, L, cf, alpha, minv, beta, st, red, nblk_alloc, N64, NF, tid);
  }
  // the last workgroup to finish takes the step's scalars from the column totals
  __shared__ double tot[5 * kMaxCols];
  if (!last_block_ticket(red.cnt_cols, (uint32_t)G)) return;
  const int nc = K + nt;
  for (int e = tid; e < nc * 5; e += kWsThreads) {
    const int cc = e / 5, v = e - (e / 5) * 5;
    tot[v * nc + cc] = load_agent(&red.colsum[e]);
  }
  if (tid == 0) store_agent(red.cnt_cols, 0u);
  __syncthreads();
  finish_fused(st, tot, nc, ctl);
}

bool conv_ws_ok(const ConvDims& cd) {
  // kernel sides 1, 5, 9: the staged region then starts on a multiple of
  // four columns (2c = ks - 1), and with W a multiple of four every 16-byte
  // vector of it is aligned
  if (cd.fp64 || cd.perm != 0 || (cd.ks != 1 && cd.ks != 5 && cd.ks != 9) || cd.W % 4 != 0) return false;
  if (cd.K + cd.nt > kMaxCols) return false;
  if ((4 * (int64_t)cd.nt + cd.K) * cd.tilesX * cd.tilesY >= ((int64_t)1 << 30)) return false;
  if (cd.D >= ((int64_t)1 << 28)) return false;  // 32-bit pixel offsets within a column
  // the staged regions of both unit kinds wrap at most one period
  const int c = (cd.ks - 1) / 2;
  const int trf = ((kConvTile + 2 * c + 3) / 4) * 4, trd = ((kConvTile / 2 + 2 * c + 3) / 4) * 4;
  const int xw = ((cd.ks + 3 + 3) / 4) * 4;
  const int need_h = trf > trd ? trf : trd;
  const int need_w = (trf + xw - 4 - 2 * c) > (trd + xw - 4 - 2 * c) ? (trf + xw - 4 - 2 * c) : (trd + xw - 4 - 2 * c);
  return cd.H >= need_h && cd.W >= need_w;
}

hipError_t conv_fused_ws(const ConvDims& cd, int grid, const float* taps, const ConvState& s0, const ConvState& s1,
                         void* X, double* xm, const float* alpha, double beta, const float* minv,
                         const ConvReduce& red, CgScalars* st, hipStream_t s) {
  if (!conv_ws_ok(cd) || grid < 1) return hipErrorInvalidValue;
  const int ntiles = cd.tilesX * cd.tilesY;
  const int64_t nblk_alloc = conv_pass_blocks(cd);
#define COFEM_WS_CASE(KS)                                                                                          \
  case KS:                                                                                                         \
    hipLaunchKernelGGL((k_conv_ws<KS>), dim3((unsigned)grid), dim3(kWsThreads), 0, s, taps, cd.H, cd.W, cd.ldD,    \
                       cd.K, cd.nt, cd.tilesX, ntiles, static_cast<const float*>(s0.P),                             \
                       static_cast<const float*>(s0.R), static_cast<const float*>(s0.Q), static_cast<float*>(X),    \
                       static_cast<float*>(s1.P), static_cast<float*>(s1.R), static_cast<float*>(s1.Q), s0.pm,      \
                       s0.rm, s0.qm, xm, s1.pm, s1.rm, s1.qm, alpha, beta, minv, red, nblk_alloc, st);              \
    break;
  switch (cd.ks) {
    COFEM_WS_CASE(1)
    COFEM_WS_CASE(5)
    COFEM_WS_CASE(9)
    default:
      return hipErrorInvalidValue;
  }
#undef COFEM_WS_CASE
  return hipGetLastError();
}

}  // namespace cofem
