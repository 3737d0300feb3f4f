// Spectral start of the convolution dictionary's E-step.
//
// With a uniform alpha = a (the first E-step of Algorithm 1, which starts
// from alpha = 1) the E-step matrix of Eq. 3, A = beta Phi^T Phi + a I, is
// block-circulant for the circular-convolution dictionary: the 2D DFT
// diagonalises it with eigenvalues
//   lambda(k1, k2) = beta |h_hat(k1, k2)|^2 + a,
//   h_hat(k1, k2)  = sum_{a,b} h[a,b] exp(-2 pi i (k1 a / H + k2 b / W))
// (a shift of the kernel only changes h_hat's phase).  The solve of the
// K + T right-hand sides B = [p_1 .. p_K | b0_1 .. b0_T] (Eq. 7) is then
//   X0 = IDFT2( DFT2(B) / lambda ),
// an O(D log D) product, the complexity Sec. 1 and Sec. 3.2 give for
// structured dictionaries.  It is formed in single precision and handed to
// the solver as its starting block; CG's own stop test (Sec. 3.2) then judges
// it and corrects what rounding left (not in the paper: a start).
//
// Transforms: two real columns travel as one complex signal z = b_c + i b_c+1.
// lambda is real and lambda(-k) = lambda(k), so the filtered inverse returns
// x_c + i x_c+1 exactly.  H and W are powers of two (at most 4096); every
// line transform is a radix-2 FFT over a 64 KiB LDS tile of 8192 complex
// values (several rows, or several columns, per workgroup):
//   k_spec_rows_fwd  B regenerated (probes of EM iteration t, b0), row DFTs
//                    (decimation in time from bit-reversed loads) -> Z
//   k_spec_cols      column DFTs, division by lambda, inverse column DFTs
//                    (decimation in frequency, stored from bit-reversed
//                    positions) in place in Z
//   k_spec_rows_inv  inverse row DFTs, 1/(H W), real and imaginary parts to
//                    the two columns of the start block (probe columns in the
//                    state's precision, mean columns float64).
// Z holds ceil((K + T)/2) complex images of H x W (pair j at j * D).
#include "cofem_internal.h"

namespace cofem {

namespace {

constexpr int kSpecThreads = 256;
constexpr int kSpecLgTile = 13;
constexpr int kSpecTile = 1 << kSpecLgTile;  // complex values per workgroup tile

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int bit_reverse(int i, int lg) {
  return lg > 0 ? (int)(__brev((unsigned)i) >> (32 - lg)) : 0;
}

// Radix-2 stages over the lines of the tile: line r (length 2^lg) at r << lg,
// nlines << (lg - 1) butterflies per stage spread over the workgroup.
// tw[i] = exp(-2 pi i i / 2^nmax_lg); the stage of span 2^s uses
// w = exp(-+ 2 pi i k / 2^s) = tw[k << (nmax_lg - s)] (conjugated for INV).
// Decimation in time: bit-reversed input, natural output.
template <bool INV>
__device__ void fft_dit(float2* x, int lg, int nlines, const float2* __restrict__ tw, int nmax_lg) {
  const int nb = nlines << (lg - 1);
  for (int s = 1; s <= lg; ++s) {
    const int half = 1 << (s - 1);
    for (int b = threadIdx.x; b < nb; b += kSpecThreads) {
      const int r = b >> (lg - 1), k2 = b & ((1 << (lg - 1)) - 1);
      const int k = k2 & (half - 1);
      const int i0 = (r << lg) + ((k2 >> (s - 1)) << s) + k, i1 = i0 + half;
      float2 w = tw[k << (nmax_lg - s)];
      if (INV) w.y = -w.y;
      const float2 t = cmul(w, x[i1]);
      const float2 u = x[i0];
      x[i0] = make_float2(u.x + t.x, u.y + t.y);
      x[i1] = make_float2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
}

// Decimation in frequency: natural input, bit-reversed output.
template <bool INV>
__device__ void fft_dif(float2* x, int lg, int nlines, const float2* __restrict__ tw, int nmax_lg) {
  const int nb = nlines << (lg - 1);
  for (int s = lg; s >= 1; --s) {
    const int half = 1 << (s - 1);
    for (int b = threadIdx.x; b < nb; b += kSpecThreads) {
      const int r = b >> (lg - 1), k2 = b & ((1 << (lg - 1)) - 1);
      const int k = k2 & (half - 1);
      const int i0 = (r << lg) + ((k2 >> (s - 1)) << s) + k, i1 = i0 + half;
      float2 w = tw[k << (nmax_lg - s)];
      if (INV) w.y = -w.y;
      const float2 a = x[i0], c = x[i1];
      x[i0] = make_float2(a.x + c.x, a.y + c.y);
      x[i1] = cmul(make_float2(a.x - c.x, a.y - c.y), w);
    }
    __syncthreads();
  }
}

// Column c of B at pixel pix (c >= K + T: the zero padding of an odd count).
__device__ __forceinline__ float b_value(int c, int64_t pix, int K, int nt, int64_t ldD, uint64_t seed, int t,
                                         const double* __restrict__ b0) {
  if (c < K) return probe_sign(seed, (uint32_t)t, (uint32_t)c, (uint64_t)pix);
  if (c < K + nt) return (float)b0[(int64_t)(c - K) * ldD + pix];
  return 0.0f;
}

template <typename TP>
__device__ __forceinline__ void x_store(int c, int64_t pix, float v, int K, int nt, int64_t ldD, TP* __restrict__ X,
                                        double* __restrict__ xm) {
  if (c < K)
    X[(int64_t)c * ldD + pix] = (TP)v;
  else if (c < K + nt)
    xm[(int64_t)(c - K) * ldD + pix] = (double)v;
}

}  // namespace

// tw[i] = exp(-2 pi i i / 2^nmax_lg), i < max(1, 2^(nmax_lg - 1)), from
// float64 sincospi.
__global__ void k_spec_twiddle(int nmax_lg, float2* __restrict__ tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = nmax_lg > 0 ? 1 << (nmax_lg - 1) : 1;
  if (i >= n) return;
  double sn, cs;
  sincospi(-2.0 * (double)i / (double)(1 << nmax_lg), &sn, &cs);
  tw[i] = make_float2((float)cs, (float)sn);
}

// g[k1 W + k2] = |h_hat(k1, k2)|^2 in float64, stored as float.  The kernel's
// DFT is separable in its phase factors: h_hat = sum_a e_a sum_b h[a,b] f_b
// with e_a = exp(-2 pi i k1 a / H), f_b = exp(-2 pi i k2 b / W).
__global__ void k_spec_gram(int H, int W, int ks, const float* __restrict__ taps, float* __restrict__ g) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)H * W) return;
  const int k1 = (int)(idx / W), k2 = (int)(idx - (idx / W) * W);
  double fr[9], fi[9];
  for (int b = 0; b < ks; ++b) {
    const int64_t m = ((int64_t)k2 * b) % W;
    sincospi(-2.0 * (double)m / (double)W, &fi[b], &fr[b]);
  }
  double re = 0.0, im = 0.0;
  for (int a = 0; a < ks; ++a) {
    double ir = 0.0, ii = 0.0;
    for (int b = 0; b < ks; ++b) {
      const double h = (double)taps[a * ks + b];
      ir += h * fr[b];
      ii += h * fi[b];
    }
    double es, ec;
    const int64_t m = ((int64_t)k1 * a) % H;
    sincospi(-2.0 * (double)m / (double)H, &es, &ec);
    re += ec * ir - es * ii;
    im += ec * ii + es * ir;
  }
  g[idx] = (float)(re * re + im * im);
}

__global__ __launch_bounds__(kSpecThreads) void k_spec_rows_fwd(int H, int W, int lgW, int nmax_lg, int64_t D,
                                                                int64_t ldD, int K, int nt, uint64_t seed, int t,
                                                                const double* __restrict__ b0,
                                                                const float2* __restrict__ tw,
                                                                float2* __restrict__ Z) {
  __shared__ float2 x[kSpecTile];
  const int R = kSpecTile >> lgW;  // rows in the tile
  const int u0 = blockIdx.x * R, j = blockIdx.y;
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int r = e >> lgW, v = e & (W - 1), u = u0 + r;
    float2 z = make_float2(0.0f, 0.0f);
    if (u < H) {
      const int64_t pix = (int64_t)u * W + v;
      z.x = b_value(2 * j, pix, K, nt, ldD, seed, t, b0);
      z.y = b_value(2 * j + 1, pix, K, nt, ldD, seed, t, b0);
    }
    x[(r << lgW) + bit_reverse(v, lgW)] = z;
  }
  __syncthreads();
  if (lgW > 0) fft_dit<false>(x, lgW, R, tw, nmax_lg);
  float2* zj = Z + (int64_t)j * D;
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int r = e >> lgW, u = u0 + r;
    if (u < H) zj[(int64_t)u * W + (e & (W - 1))] = x[e];
  }
}

// Column block: C = kSpecTile / H adjacent columns of pair j, column cc at
// cc << lgH in the tile.  Loads and stores walk a row's C values with
// consecutive threads.
__global__ __launch_bounds__(kSpecThreads) void k_spec_cols(int H, int W, int lgH, int nmax_lg, int64_t D,
                                                            const float* __restrict__ g, double beta, double a0,
                                                            const float2* __restrict__ tw, float2* __restrict__ Z) {
  __shared__ float2 x[kSpecTile];
  const int lgC = kSpecLgTile - lgH, C = 1 << lgC;
  const int v0 = blockIdx.x * C, j = blockIdx.y;
  float2* zj = Z + (int64_t)j * D;
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int u = e >> lgC, cc = e & (C - 1), v = v0 + cc;
    x[(cc << lgH) + bit_reverse(u, lgH)] = v < W ? zj[(int64_t)u * W + v] : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  if (lgH > 0) fft_dit<false>(x, lgH, C, tw, nmax_lg);
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int k1 = e >> lgC, cc = e & (C - 1), v = v0 + cc;
    if (v < W) {
      const float s = (float)(1.0 / (beta * (double)g[(int64_t)k1 * W + v] + a0));
      const int i = (cc << lgH) + k1;
      x[i] = make_float2(x[i].x * s, x[i].y * s);
    }
  }
  __syncthreads();
  if (lgH > 0) fft_dif<true>(x, lgH, C, tw, nmax_lg);
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int u = e >> lgC, cc = e & (C - 1), v = v0 + cc;
    if (v < W) zj[(int64_t)u * W + v] = x[(cc << lgH) + bit_reverse(u, lgH)];
  }
}

template <typename TP>
__global__ __launch_bounds__(kSpecThreads) void k_spec_rows_inv(int H, int W, int lgW, int nmax_lg, int64_t D,
                                                                int64_t ldD, int K, int nt, float scale,
                                                                const float2* __restrict__ tw,
                                                                const float2* __restrict__ Z, TP* __restrict__ X,
                                                                double* __restrict__ xm) {
  __shared__ float2 x[kSpecTile];
  const int R = kSpecTile >> lgW;
  const int u0 = blockIdx.x * R, j = blockIdx.y;
  const float2* zj = Z + (int64_t)j * D;
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int r = e >> lgW, u = u0 + r;
    x[e] = u < H ? zj[(int64_t)u * W + (e & (W - 1))] : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  if (lgW > 0) fft_dif<true>(x, lgW, R, tw, nmax_lg);
  for (int e = threadIdx.x; e < kSpecTile; e += kSpecThreads) {
    const int r = e >> lgW, v = e & (W - 1), u = u0 + r;
    if (u < H) {
      const int64_t pix = (int64_t)u * W + v;
      const float2 z = x[(r << lgW) + bit_reverse(v, lgW)];
      x_store(2 * j, pix, z.x * scale, K, nt, ldD, X, xm);
      x_store(2 * j + 1, pix, z.y * scale, K, nt, ldD, X, xm);
    }
  }
}

namespace {
int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}
}  // namespace

bool conv_spectral_ok(int H, int W) {
  const int lh = log2_exact(H), lw = log2_exact(W);
  return H >= 1 && W >= 1 && lh >= 0 && lw >= 0 && H <= kSpecMaxSide && W <= kSpecMaxSide;
}

int64_t conv_spectral_pairs(const ConvDims& cd) { return (cd.K + cd.nt + 1) / 2; }

int64_t conv_spectral_twiddles(const ConvDims& cd) {
  const int n = cd.H > cd.W ? cd.H : cd.W;
  return n > 1 ? n / 2 : 1;
}

hipError_t conv_spectral_tables(const ConvDims& cd, const float* taps, float* g, float2* tw, hipStream_t s) {
  if (!conv_spectral_ok(cd.H, cd.W)) return hipErrorInvalidValue;
  const int nmax_lg = log2_exact(cd.H > cd.W ? cd.H : cd.W);
  const int64_t ntw = conv_spectral_twiddles(cd);
  hipLaunchKernelGGL(k_spec_twiddle, dim3((unsigned)((ntw + 255) / 256)), dim3(256), 0, s, nmax_lg, tw);
  hipLaunchKernelGGL(k_spec_gram, dim3((unsigned)((cd.D + 255) / 256)), dim3(256), 0, s, cd.H, cd.W, cd.ks, taps,
                     g);
  return hipGetLastError();
}

hipError_t conv_spectral_start(const ConvDims& cd, uint64_t seed, int t, const double* b0, const float* g,
                               const float2* tw, double beta, double a0, float2* Z, void* X, double* xm,
                               hipStream_t s) {
  if (!conv_spectral_ok(cd.H, cd.W) || cd.perm != 0) return hipErrorInvalidValue;
  const int lgH = log2_exact(cd.H), lgW = log2_exact(cd.W);
  const int nmax_lg = lgH > lgW ? lgH : lgW;
  const unsigned pairs = (unsigned)conv_spectral_pairs(cd);
  const int R = kSpecTile >> lgW, C = kSpecTile >> lgH;
  const dim3 grow((unsigned)((cd.H + R - 1) / R), pairs), gcol((unsigned)((cd.W + C - 1) / C), pairs);
  hipLaunchKernelGGL(k_spec_rows_fwd, grow, dim3(kSpecThreads), 0, s, cd.H, cd.W, lgW, nmax_lg, cd.D, cd.ldD, cd.K,
                     cd.nt, seed, t, b0, tw, Z);
  hipLaunchKernelGGL(k_spec_cols, gcol, dim3(kSpecThreads), 0, s, cd.H, cd.W, lgH, nmax_lg, cd.D, g, beta, a0, tw,
                     Z);
  const float scale = (float)(1.0 / (double)cd.D);
  if (cd.fp64)
    hipLaunchKernelGGL(k_spec_rows_inv<double>, grow, dim3(kSpecThreads), 0, s, cd.H, cd.W, lgW, nmax_lg, cd.D,
                       cd.ldD, cd.K, cd.nt, scale, tw, Z, static_cast<double*>(X), xm);
  else
    hipLaunchKernelGGL(k_spec_rows_inv<float>, grow, dim3(kSpecThreads), 0, s, cd.H, cd.W, lgW, nmax_lg, cd.D,
                       cd.ldD, cd.K, cd.nt, scale, tw, Z, static_cast<float*>(X), xm);
  return hipGetLastError();
}

}  // namespace cofem
