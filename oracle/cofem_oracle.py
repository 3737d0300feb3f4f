"""Plain FP64 CPU oracle of covariance-free EM (CoFEM) for sparse Bayesian learning.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the HIP product path.

Paper: Lin, Song, Bilgic, Ba, "High-Dimensional Sparse Bayesian Learning without
Covariance Matrices" (arXiv 2202.12808).  Every function below names the passage
it follows.  Everything is float64; problem data (Phi or taps, y, alpha) is
whatever the caller passes, upcast to float64.

Readings of the paper taken here (each is also a row of the design notes):

* The system matrix is A = beta*Phi^T*Phi + diag(alpha) (Eq. 3, Eq. 5, Eq. 7,
  Algorithm 1); the CG subsection writes A without beta, read as a typo.
* CG stops when the joint Frobenius ratio ||R||_F/||B||_F of the *recursively
  updated* residual falls below eps, or after U iterations (Sec. 3.2); every
  column runs the same number of iterations.  X0 = 0.
* Probes are redrawn at every EM iteration (Algorithm 1 draws them inside the
  loop) from a counter-based SplitMix64 stream: see ``rademacher_probes``.
* Column order of B is [p_1 .. p_K | beta*Phi^T*y] (Eq. 7): mu is column K.
* The M-step denominator mu^2 + s can be <= 0 for finite K (s is a Monte-Carlo
  estimate); it is floored at 1/alpha_max with alpha_max = 1e10, so
  alpha <- 1 / max(mu^2 + s, 1/alpha_max).  Exact EM never hits the floor.
* The structured dictionary is a 2D circular convolution with an odd k x k
  kernel centred at ((kh-1)/2, (kw-1)/2); N = D = H*W; pixel index j = u*W + v.
* The DCT dictionary of Sec. 4 is Phi = S C^T with C the orthonormal DCT-II
  matrix (C^T is the inverse DCT) over a length-D signal and S the selection
  of N distinct observed samples (``DctMaskOperator``).

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
closed forms, brute force, textbook factorizations or the published SplitMix64
output stream -- never against its own formula retyped.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

ALPHA_MAX_DEFAULT = 1e10

# ---------------------------------------------------------------------------
# Counter-based SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
# number generators", OOPSLA 2014).  The n-th output (n = 1, 2, ...) for seed s
# is mix64(s + n * GAMMA mod 2^64).
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (variant 13 of Stafford's mix) on uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_stream(seed: int, counters: np.ndarray) -> np.ndarray:
    """Output number ``counters`` (1-based) of the SplitMix64 stream of ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + c * _GAMMA
    return splitmix64_mix(state)


def rademacher_probes(seed: int, t: int, K: int, D: int) -> np.ndarray:
    """Probe matrix P_t in {+1,-1}^{D x K} of EM iteration t (Sec. 3.1, Eq. 6;
    Algorithm 1 draws p_1..p_K inside the EM loop).

    Sign of entry (j, k): take the 64-bit word number
        i = (t << 48) | (k << 32) | (j >> 6)
    of the SplitMix64 stream of ``seed`` (1-based: counter i + 1); bit (j & 63)
    of that word selects the sign, 0 -> +1, 1 -> -1.  t < 2^16, k < 2^16,
    j < 2^38.
    """
    if not (0 <= t < (1 << 16) and 0 <= K <= (1 << 16) and 0 <= D < (1 << 38)):
        raise ValueError("probe index out of range")
    j = np.arange(D, dtype=np.uint64)
    out = np.empty((D, K), dtype=np.float64)
    for k in range(K):
        idx = (np.uint64(t) << np.uint64(48)) | (np.uint64(k) << np.uint64(32)) | (j >> np.uint64(6))
        words = splitmix64_stream(seed, idx + np.uint64(1))
        bits = (words >> (j & np.uint64(63))) & np.uint64(1)
        out[:, k] = 1.0 - 2.0 * bits.astype(np.float64)
    return out


# ---------------------------------------------------------------------------
# Dictionaries: something that applies Phi and Phi^T (Sec. 3.2: CG only needs
# a way to apply A, i.e. Phi and Phi^T).
# ---------------------------------------------------------------------------
class DenseOperator:
    """Dense dictionary Phi in R^{N x D} (Eq. 1)."""

    def __init__(self, phi: np.ndarray):
        self.phi = np.asarray(phi, dtype=np.float64)
        self.N, self.D = self.phi.shape

    def apply(self, v: np.ndarray) -> np.ndarray:
        return self.phi @ v

    def apply_t(self, w: np.ndarray) -> np.ndarray:
        return self.phi.T @ w

    def column_norms_sq(self) -> np.ndarray:
        return np.einsum("nd,nd->d", self.phi, self.phi)


class ConvOperator:
    """2D circular convolution dictionary (a structured Phi with fast apply,
    Sec. 1 and Sec. 3.2).

    (Phi z)[u, v] = sum_{a,b} h[a, b] * z[(u - a + ch) mod H, (v - b + cw) mod W]
    with ch = (kh - 1)/2, cw = (kw - 1)/2; Phi^T is the matching circular
    correlation.  Vectors are images flattened row-major (j = u*W + v).
    The sum over taps is evaluated per image by scipy.ndimage's wrap-mode
    convolve / correlate (a library stencil: the plain definition, in C),
    one thread per column.
    """

    def __init__(self, taps: np.ndarray, H: int, W: int):
        self.taps = np.asarray(taps, dtype=np.float64)
        kh, kw = self.taps.shape
        if kh % 2 == 0 or kw % 2 == 0:
            raise ValueError("kernel sides must be odd")
        self.H, self.W = int(H), int(W)
        self.N = self.D = self.H * self.W
        self.ch, self.cw = (kh - 1) // 2, (kw - 1) // 2

    def _map(self, fn, v):
        import scipy.ndimage as nd

        v = np.asarray(v, dtype=np.float64)
        one = v.ndim == 1
        cols = v.reshape(self.D, -1)
        f = getattr(nd, fn)

        def one_col(k):
            return f(cols[:, k].reshape(self.H, self.W), self.taps, mode="wrap").reshape(self.D)

        m = cols.shape[1]
        if m == 1:
            out = one_col(0)[:, None]
        else:
            out = np.stack(list(_pool().map(one_col, range(m))), axis=1)
        return out[:, 0] if one else out

    def apply(self, v: np.ndarray) -> np.ndarray:
        return self._map("convolve", v)

    def apply_t(self, w: np.ndarray) -> np.ndarray:
        return self._map("correlate", w)

    def column_norms_sq(self) -> np.ndarray:
        return np.full(self.D, float(np.sum(self.taps * self.taps)))


class ConvOperatorFFT:
    """The circular convolution dictionary of ``ConvOperator`` applied through
    the convolution theorem: with the taps placed on the H x W grid so that
    tap (ch, cw) sits at the origin, Phi is multiplication of the 2D DFT by
    the kernel's DFT h_hat, Phi^T by conj(h_hat), and Phi^T Phi (the only
    product CG needs, Sec. 3.2) by |h_hat|^2 -- one forward and one inverse
    real transform per column instead of two k x k stencils.  scipy.fft does
    the transforms (a library FFT used as a step), over the host's threads.
    """

    def __init__(self, taps: np.ndarray, H: int, W: int):
        import scipy.fft as sf

        self.taps = np.asarray(taps, dtype=np.float64)
        kh, kw = self.taps.shape
        if kh % 2 == 0 or kw % 2 == 0:
            raise ValueError("kernel sides must be odd")
        self.H, self.W = int(H), int(W)
        self.N = self.D = self.H * self.W
        ch, cw = (kh - 1) // 2, (kw - 1) // 2
        kern = np.zeros((self.H, self.W))
        for a in range(kh):
            for b in range(kw):
                kern[(a - ch) % self.H, (b - cw) % self.W] += self.taps[a, b]
        self.h_hat = sf.rfft2(kern)
        self.gram_hat = (self.h_hat * np.conj(self.h_hat)).real
        import os
        self.workers = max(1, min(16, os.cpu_count() or 1))

    def _filter(self, v, spec):
        import scipy.fft as sf

        v = np.asarray(v, dtype=np.float64)
        one = v.ndim == 1
        img = v.reshape(self.H, self.W, -1)
        f = sf.rfft2(img, axes=(0, 1), workers=self.workers)
        f *= spec[:, :, None]
        out = sf.irfft2(f, s=(self.H, self.W), axes=(0, 1), workers=self.workers).reshape(self.D, -1)
        return out[:, 0] if one else out

    def apply(self, v: np.ndarray) -> np.ndarray:
        return self._filter(v, self.h_hat)

    def apply_t(self, w: np.ndarray) -> np.ndarray:
        return self._filter(w, np.conj(self.h_hat))

    def gram(self, v: np.ndarray) -> np.ndarray:
        """Phi^T Phi v."""
        return self._filter(v, self.gram_hat)

    def column_norms_sq(self) -> np.ndarray:
        return np.full(self.D, float(np.sum(self.taps ** 2)))

    def solve_shifted(self, B: np.ndarray, beta: float, a: float) -> np.ndarray:
        """X = (beta Phi^T Phi + a I)^-1 B: with a uniform alpha = a the matrix
        A of Eq. 3 is block-circulant (Phi^T Phi is a circular convolution), so
        the 2D DFT diagonalises it with eigenvalues beta |h_hat|^2 + a and the
        solve is a division in the Fourier domain (not in the paper: the exact
        start of the spectral form)."""
        if not a > 0.0:
            raise ValueError("a must be positive")
        return self._filter(B, 1.0 / (beta * self.gram_hat + float(a)))


class DctMaskOperator:
    """Inverse DCT followed by an undersampling mask (the structured dictionary
    of Sec. 4, "Structured Dictionary"): Phi = S C^T in R^{N x D}.

    C is the D x D orthonormal DCT-II matrix,
        C[k, n] = c_k cos(pi (2n + 1) k / (2D)),  c_0 = sqrt(1/D), c_k = sqrt(2/D),
    so C^T (the orthonormal DCT-III) is the inverse DCT, and S keeps the N
    observed samples ``rows`` (distinct indices into the length-D signal):
    (Phi z)_i = (C^T z)[rows[i]].  z holds DCT coefficients.  The paper fixes
    neither the DCT type, its normalisation nor how the samples are chosen;
    with the orthonormal type II, Phi Phi^T = I_N.  apply / apply_t call
    scipy.fft's idct / dct (a library transform: the definition above, in
    O(D log D)), one call for all columns.
    """

    def __init__(self, rows: np.ndarray, D: int):
        rows = np.asarray(rows, dtype=np.int64)
        self.D = int(D)
        if rows.ndim != 1 or rows.size == 0 or rows.min() < 0 or rows.max() >= self.D:
            raise ValueError("rows must be indices into [0, D)")
        if np.unique(rows).size != rows.size:
            raise ValueError("rows must be distinct")
        self.rows = rows
        self.N = rows.size

    def apply(self, v: np.ndarray) -> np.ndarray:
        import scipy.fft as sf

        v = np.asarray(v, dtype=np.float64)
        return sf.idct(v, type=2, norm="ortho", axis=0)[self.rows]

    def apply_t(self, w: np.ndarray) -> np.ndarray:
        import scipy.fft as sf

        w = np.asarray(w, dtype=np.float64)
        full = np.zeros((self.D,) + w.shape[1:])
        full[self.rows] = w
        return sf.dct(full, type=2, norm="ortho", axis=0)

    def column_norms_sq(self) -> np.ndarray:
        """||Phi e_k||^2 = sum over observed samples n of C[k, n]^2, from the
        cosine definition (O(N D): small problems)."""
        k = np.arange(self.D, dtype=np.float64)[:, None]
        c2 = np.full(self.D, 2.0 / self.D)
        c2[0] = 1.0 / self.D
        out = np.zeros(self.D)
        for lo in range(0, self.N, 1024):
            n = self.rows[lo:lo + 1024].astype(np.float64)[None, :]
            out += np.sum(np.cos(np.pi * (2.0 * n + 1.0) * k / (2.0 * self.D)) ** 2, axis=1)
        return c2 * out


_POOL = None


def _pool():
    global _POOL
    if _POOL is None:
        import os
        from concurrent.futures import ThreadPoolExecutor

        _POOL = ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1)))
    return _POOL


def make_apply_A(op, beta: float, alpha: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    """v -> A v with A = beta*Phi^T*Phi + diag(alpha) (Eq. 5, Eq. 7)."""
    alpha = np.asarray(alpha, dtype=np.float64)

    gram = getattr(op, "gram", None)

    def apply_A(V):
        V = np.asarray(V, dtype=np.float64)
        av = alpha[:, None] * V if V.ndim == 2 else alpha * V
        g = gram(V) if gram is not None else op.apply_t(op.apply(V))
        return beta * g + av

    return apply_A


# ---------------------------------------------------------------------------
# Multi-right-hand-side conjugate gradient (Sec. 3.2; Hestenes & Stiefel 1952,
# Shewchuk 1994), mat-vecs replaced by mat-mats.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class CGInfo:
    iters: int
    converged: bool
    rel_resid: float          # recursive ||R||_F / ||B||_F at exit
    history: list             # recursive ratio before each iteration


def cg_solve(apply_A, B: np.ndarray, tol: float, max_iter: int,
             fixed_iters: Optional[int] = None, stop_rule: str = "frobenius"):
    """Solve A X = B column by column with plain CG from X0 = 0.

    Column c keeps its own step a_c = rho_c / (p_c^T A p_c) and direction update
    b_c = rho'_c / rho_c.  With the default stop rule the whole block stops
    once sqrt(sum_c rho_c) / ||B||_F < tol (rho_c = ||r_c||^2, recursive
    residual) or after ``max_iter`` iterations.  With ``stop_rule =
    "per_column"`` column c is finished once ||r_c|| / ||b_c|| < tol (a zero
    column from the start): it takes no further step (a_c = 0, its x_c and r_c
    stay as they are, its direction is reset to r_c), and the block stops when
    every column is finished or at the cap.  With ``fixed_iters`` set, exactly
    that many iterations run and the tolerance is ignored.  A column whose rho
    or p^T A p is exactly zero takes a zero step.
    """
    per_col = _check_stop_rule(stop_rule)
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B)
    R = B.copy()
    P = R.copy()
    rho = np.einsum("dc,dc->c", R, R)
    bb = rho.copy()
    nB = math.sqrt(float(rho.sum()))
    hist = []
    done = np.zeros(B.shape[1], dtype=bool)
    if nB == 0.0:
        return X, CGInfo(0, True, 0.0, hist)
    limit = fixed_iters if fixed_iters is not None else max_iter
    it = 0
    while it < limit:
        ratio = math.sqrt(float(rho.sum())) / nB
        hist.append(ratio)
        if fixed_iters is None:
            if per_col:
                done |= (bb == 0.0) | (np.sqrt(rho) < tol * np.sqrt(bb))
                if done.all():
                    break
            elif ratio < tol:
                break
        Q = apply_A(P)
        gam = np.einsum("dc,dc->c", P, Q)
        a = np.divide(rho, gam, out=np.zeros_like(rho), where=gam != 0.0)
        a[done] = 0.0
        X += a * P
        R -= a * Q
        rho_new = np.einsum("dc,dc->c", R, R)
        b = np.divide(rho_new, rho, out=np.zeros_like(rho), where=rho != 0.0)
        b[done] = 0.0
        P = R + b * P
        rho = rho_new
        it += 1
    ratio = math.sqrt(float(rho.sum())) / nB
    if per_col and fixed_iters is None:
        done |= (bb == 0.0) | (np.sqrt(rho) < tol * np.sqrt(bb))
        return X, CGInfo(it, bool(done.all()), ratio, hist)
    return X, CGInfo(it, ratio < tol, ratio, hist)


def _check_stop_rule(stop_rule: str) -> bool:
    if stop_rule not in ("frobenius", "per_column"):
        raise ValueError(f"unknown stop rule {stop_rule!r}")
    return stop_rule == "per_column"


def pcg_solve(apply_A, B: np.ndarray, tol: float, max_iter: int, minv: Optional[np.ndarray] = None,
              X0: Optional[np.ndarray] = None, fixed_iters: Optional[int] = None,
              stop_rule: str = "frobenius"):
    """Preconditioned CG from a starting block (not in the paper: the learned
    and warm-started forms).  M^-1 = diag(minv) (a length-D positive vector,
    the same for every column; None is the identity), X0 the starting block
    (None is zero).  Column c: r = b - A x0, z = M^-1 r, p = z,
    rho = r^T z; per step a = rho / (p^T A p), x += a p, r -= a q,
    z = M^-1 r, rho' = r^T z, p = z + (rho'/rho) p.  The stop test is the
    solve's own (Sec. 3.2): sqrt(sum_c ||r_c||^2) / ||B||_F < tol on the
    recursively updated (unpreconditioned) residual, checked before every
    iteration, or the cap; with ``stop_rule = "per_column"`` each column
    stops on its own ||r_c|| / ||b_c|| < tol as in ``cg_solve``."""
    per_col = _check_stop_rule(stop_rule)
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B) if X0 is None else np.asarray(X0, dtype=np.float64).copy()
    m = np.ones(B.shape[0]) if minv is None else np.asarray(minv, dtype=np.float64)
    R = B - apply_A(X) if X0 is not None else B.copy()
    Z = m[:, None] * R
    P = Z.copy()
    rho = np.einsum("dc,dc->c", R, Z)
    bb = np.einsum("dc,dc->c", B, B)
    nB = float(np.linalg.norm(B))
    hist = []
    done = np.zeros(B.shape[1], dtype=bool)
    if nB == 0.0:
        return X, CGInfo(0, True, 0.0, hist)
    limit = fixed_iters if fixed_iters is not None else max_iter
    it = 0
    while it < limit:
        ratio = float(np.linalg.norm(R)) / nB
        hist.append(ratio)
        if fixed_iters is None:
            if per_col:
                done |= (bb == 0.0) | (np.sqrt(np.einsum("dc,dc->c", R, R)) < tol * np.sqrt(bb))
                if done.all():
                    break
            elif ratio < tol:
                break
        Q = apply_A(P)
        gam = np.einsum("dc,dc->c", P, Q)
        a = np.divide(rho, gam, out=np.zeros_like(rho), where=gam != 0.0)
        a[done] = 0.0
        X += a * P
        R -= a * Q
        Z = m[:, None] * R
        rho_new = np.einsum("dc,dc->c", R, Z)
        b = np.divide(rho_new, rho, out=np.zeros_like(rho), where=rho != 0.0)
        b[done] = 0.0
        P = Z + b * P
        rho = rho_new
        it += 1
    ratio = float(np.linalg.norm(R)) / nB
    if per_col and fixed_iters is None:
        done |= (bb == 0.0) | (np.sqrt(np.einsum("dc,dc->c", R, R)) < tol * np.sqrt(bb))
        return X, CGInfo(it, bool(done.all()), ratio, hist)
    return X, CGInfo(it, ratio < tol, ratio, hist)


def true_relative_residual(apply_A, X: np.ndarray, B: np.ndarray) -> float:
    """||B - A X||_F / ||B||_F evaluated directly (the stop test of Sec. 3.2)."""
    R = np.asarray(B, dtype=np.float64) - apply_A(np.asarray(X, dtype=np.float64))
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(R) / nb) if nb > 0 else 0.0


# ---------------------------------------------------------------------------
# Mixed-precision form of the solve (not in the paper): classical iterative
# refinement (Wilkinson 1963; Moler 1967) around the CG solve of Sec. 3.2.  The
# outer residual B - A X uses the problem's own operator; every inner
# correction solve A_in D = R uses a lower-precision operator (for example
# Phi rounded to bfloat16) and stops at a relative tolerance tol_in of its own
# right-hand side.  The outer loop stops on the true residual.
# ---------------------------------------------------------------------------
IR_STALL = 3  # sweeps in a row without halving the best true residual


@dataclasses.dataclass
class IRInfo:
    sweeps: list        # inner CG iterations of each correction solve
    iters: int          # total inner iterations
    converged: bool     # true ratio below tol at exit
    rel_resid: float    # ||B - A X||_F / ||B||_F at exit
    history: list       # the true ratio before each sweep (and at exit)


def ir_solve(apply_A, apply_A_inner, B: np.ndarray, tol: float, tol_in: float,
             max_iter: int, max_sweeps: int, fixed_inner=None, X0: Optional[np.ndarray] = None,
             minv: Optional[np.ndarray] = None):
    """Iterative refinement: X = X0 (or 0), R = B - A X; while ||R||_F/||B||_F >= tol (and
    fewer than ``max_iter`` inner iterations and ``max_sweeps`` sweeps so far,
    and fewer than IR_STALL sweeps in a row failed to halve the best ratio --
    the true residual of refinement need not fall monotonically, and once it
    stalls its evaluation has reached its rounding floor):
    D = CG(apply_A_inner, R, tol_in, remaining budget); X += D; R = B - A X.
    With ``fixed_inner`` (a list of counts) exactly those sweeps run, each for
    exactly its count.  ``minv`` (not in the paper): the inner solves are
    ``pcg_solve`` from zero with M^-1 = diag(minv) and the same stop test."""
    B = np.asarray(B, dtype=np.float64)
    if X0 is None:
        X = np.zeros_like(B)
        R = B.copy()
    else:
        X = np.array(X0, dtype=np.float64).reshape(B.shape)
        R = B - apply_A(X)
    nB = float(np.linalg.norm(B))
    sweeps, hist = [], []
    total = 0
    best, stall = None, 0
    while True:
        ratio = float(np.linalg.norm(R)) / nB if nB > 0.0 else 0.0
        hist.append(ratio)
        if best is None:
            best = ratio
        elif ratio < 0.5 * best:
            best, stall = ratio, 0
        else:
            stall += 1
        if fixed_inner is not None:
            if len(sweeps) == len(fixed_inner):
                break
        elif (ratio < tol or total >= max_iter or len(sweeps) >= max_sweeps
              or stall >= IR_STALL):
            break
        n = None if fixed_inner is None else int(fixed_inner[len(sweeps)])
        if minv is None:
            Dx, info = cg_solve(apply_A_inner, R, tol_in, max_iter - total, fixed_iters=n)
        else:
            Dx, info = pcg_solve(apply_A_inner, R, tol_in, max_iter - total, minv=minv, fixed_iters=n)
        X += Dx
        total += info.iters
        sweeps.append(info.iters)
        R = B - apply_A(X)
    return X, IRInfo(sweeps, total, ratio < tol, ratio, hist)


# ---------------------------------------------------------------------------
# Simplified E-step, diagonal estimate and M-step (Sec. 3.1, Algorithm 1)
# ---------------------------------------------------------------------------
def diag_estimate(P: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Rademacher diagonal estimate s = (1/K) sum_k p_k (.) x_k  (Eq. 6, with
    x_k = Sigma p_k the solution of A x = p_k)."""
    K = P.shape[1]
    return np.sum(np.asarray(P, np.float64) * np.asarray(X, np.float64), axis=1) / K


def diag_estimate_ratio(P: np.ndarray, MP: np.ndarray) -> np.ndarray:
    """General diagonal-estimation rule of the Proposition (Sec. 3.1):
    s = (sum_k p_k (.) M p_k) ./ (sum_k p_k (.) p_k), for any zero-mean probes."""
    P = np.asarray(P, np.float64)
    return np.sum(P * np.asarray(MP, np.float64), axis=1) / np.sum(P * P, axis=1)


def mstep(mu: np.ndarray, s: np.ndarray, alpha_max: float = ALPHA_MAX_DEFAULT):
    """alpha <- 1 ./ (mu (.) mu + s)  (Eq. 4 with s for diag(Sigma), Eq. 8),
    denominator floored at 1/alpha_max.  Returns (alpha, number floored)."""
    denom = np.asarray(mu, np.float64) ** 2 + np.asarray(s, np.float64)
    floor = 1.0 / alpha_max
    clamped = denom < floor
    return 1.0 / np.maximum(denom, floor), int(np.count_nonzero(clamped))


@dataclasses.dataclass
class EStepResult:
    mu: np.ndarray
    s: np.ndarray
    X: np.ndarray
    P: np.ndarray
    cg: CGInfo


def cofem_estep(op, b0: np.ndarray, beta: float, alpha: np.ndarray, K: int,
                tol: float, max_iter: int, seed: int, t: int,
                fixed_iters: Optional[int] = None, stop_rule: str = "frobenius") -> EStepResult:
    """One simplified E-step of Algorithm 1 at EM iteration t: draw probes,
    form B = [P | b0] (Eq. 7), solve A X = B by CG, read mu (last column) and
    s (Eq. 6)."""
    D = op.D
    P = rademacher_probes(seed, t, K, D)
    B = np.concatenate([P, np.asarray(b0, np.float64)[:, None]], axis=1)
    X, info = cg_solve(make_apply_A(op, beta, alpha), B, tol, max_iter, fixed_iters, stop_rule)
    mu = X[:, K].copy()
    s = diag_estimate(P, X[:, :K])
    return EStepResult(mu=mu, s=s, X=X, P=P, cg=info)


def cofem_estep_ir(op, op_inner, b0: np.ndarray, beta: float, alpha: np.ndarray, K: int,
                   tol: float, tol_in: float, max_iter: int, max_sweeps: int, seed: int, t: int,
                   fixed_inner=None, mu0=None, d0=None, minv=None):
    """The E-step of Algorithm 1 with the solve done by ``ir_solve``: outer
    residual with ``op`` (the problem's Phi), inner corrections with
    ``op_inner`` (a lower-precision Phi).  With mu0 / d0 the refinement starts
    from X0 = [d0 (.) p_1 .. d0 (.) p_K | mu0] (the warm start of
    ``cofem_estep_pcg``; None entries zero).  ``minv``: the inner solves'
    diagonal preconditioner (``ir_solve``).  Returns (EStepResult, IRInfo)."""
    D = op.D
    P = rademacher_probes(seed, t, K, D)
    B = np.concatenate([P, np.asarray(b0, np.float64)[:, None]], axis=1)
    X0 = None
    if mu0 is not None or d0 is not None:
        X0 = np.zeros_like(B)
        if d0 is not None:
            X0[:, :K] = np.asarray(d0, np.float64)[:, None] * P
        if mu0 is not None:
            X0[:, K] = np.asarray(mu0, np.float64)
    X, info = ir_solve(make_apply_A(op, beta, alpha), make_apply_A(op_inner, beta, alpha), B, tol,
                       tol_in, max_iter, max_sweeps, fixed_inner, X0, minv=minv)
    mu = X[:, K].copy()
    s = diag_estimate(P, X[:, :K])
    cg = CGInfo(info.iters, info.converged, info.rel_resid, info.history)
    return EStepResult(mu=mu, s=s, X=X, P=P, cg=cg), info


def spectral_operator(op) -> "ConvOperatorFFT":
    """The Fourier-domain form of a circular-convolution dictionary."""
    if isinstance(op, ConvOperatorFFT):
        return op
    if isinstance(op, ConvOperator):
        return ConvOperatorFFT(op.taps, op.H, op.W)
    raise ValueError("the spectral start needs a circular-convolution dictionary")


def cofem_estep_pcg(op, b0: np.ndarray, beta: float, alpha: np.ndarray, K: int, tol: float, max_iter: int,
                    seed: int, t: int, minv=None, mu0=None, d0=None, fixed_iters=None,
                    stop_rule: str = "frobenius", spectral: bool = False) -> EStepResult:
    """The E-step of Algorithm 1 solved by ``pcg_solve``: M^-1 = diag(minv);
    starting block X0 = [d0 (.) p_1 .. d0 (.) p_K | mu0] (a warm start for
    the probe solves x_k ~ Sigma p_k from a diagonal estimate d0, and for mu);
    None entries start from zero.  ``spectral`` (convolution dictionaries,
    alpha uniform): X0 = A^-1 B from ``ConvOperatorFFT.solve_shifted``
    instead, and the solve goes on from there with its own stop test."""
    D = op.D
    P = rademacher_probes(seed, t, K, D)
    B = np.concatenate([P, np.asarray(b0, np.float64)[:, None]], axis=1)
    X0 = None
    if spectral:
        alpha = np.asarray(alpha, np.float64)
        if not np.all(alpha == alpha[0]):
            raise ValueError("the spectral start needs a uniform alpha")
        X0 = spectral_operator(op).solve_shifted(B, beta, float(alpha[0]))
    elif mu0 is not None or d0 is not None:
        X0 = np.zeros_like(B)
        if d0 is not None:
            X0[:, :K] = np.asarray(d0, np.float64)[:, None] * P
        if mu0 is not None:
            X0[:, K] = np.asarray(mu0, np.float64)
    X, info = pcg_solve(make_apply_A(op, beta, alpha), B, tol, max_iter, minv, X0, fixed_iters, stop_rule)
    return EStepResult(mu=X[:, K].copy(), s=diag_estimate(P, X[:, :K]), X=X, P=P, cg=info)


@dataclasses.dataclass
class CoFEMResult:
    alpha: np.ndarray
    mu: np.ndarray
    s: np.ndarray
    stats: list


def gamma_change(alpha_new: np.ndarray, alpha_old: np.ndarray) -> float:
    """Relative change of the prior variances gamma = 1/alpha over one M-step,
    ||gamma_new - gamma_old||_2 / ||gamma_new||_2: the EM-level convergence
    measure of ``cofem``'s ``em_tol`` rule (not in the paper, which runs a
    fixed T_em).  gamma rather than alpha: pruned coordinates sit at the
    1/alpha_max floor of gamma, where their Monte-Carlo flicker is invisible,
    while alpha itself would be dominated by them."""
    gn = 1.0 / np.asarray(alpha_new, np.float64)
    go = 1.0 / np.asarray(alpha_old, np.float64)
    n = float(np.linalg.norm(gn))
    return float(np.linalg.norm(gn - go)) / n if n > 0.0 else 0.0


def cofem(op, y: np.ndarray, beta: float, T_em: int, K: int, *, tol: float,
          max_iter: int, seed: int, alpha_max: float = ALPHA_MAX_DEFAULT,
          alpha0: Optional[np.ndarray] = None, t0: int = 1,
          fixed_iters=None, stop_rule: str = "frobenius",
          em_tol: Optional[float] = None, warm_start: bool = False,
          jacobi: bool = False, spectral_start: bool = False) -> CoFEMResult:
    """CovarianceFreeEM(y, Phi, beta, T_em, K) of Algorithm 1.

    alpha starts at 1 (or ``alpha0``); EM iterations are numbered t0, t0+1, ...
    (t selects the probe draw).  ``fixed_iters`` is None, an int, or a sequence
    giving the CG iteration count of each EM iteration.  Returns the final
    alpha together with mu and s of the last E-step, as Algorithm 1 does.
    With ``em_tol`` the loop also ends after the first M-step whose
    ``gamma_change`` is below em_tol (at most T_em iterations).

    ``warm_start`` / ``jacobi`` (not in the paper): each solve after the first
    starts from X0 = [max(s_prev, 0) (.) p_k | mu_prev], and/or is
    preconditioned by the inverse diagonal of A, 1 / (beta ||Phi e_j||^2 +
    alpha_j) (``cofem_estep_pcg``); the stop test is unchanged.
    ``spectral_start`` (convolution dictionaries, not in the paper): every
    E-step whose alpha is uniform (the first one from alpha = 1) starts from
    the exact solve of ``ConvOperatorFFT.solve_shifted``.
    """
    D = op.D
    alpha = np.ones(D) if alpha0 is None else np.asarray(alpha0, np.float64).copy()
    b0 = beta * op.apply_t(np.asarray(y, np.float64))
    cn = op.column_norms_sq() if jacobi else None
    stats = []
    mu = s = None
    for i in range(T_em):
        t = t0 + i
        fi = fixed_iters[i] if isinstance(fixed_iters, (list, tuple, np.ndarray)) else fixed_iters
        if warm_start or jacobi or spectral_start:
            start = dict(mu0=mu, d0=np.maximum(s, 0.0)) if (warm_start and mu is not None) else {}
            if spectral_start and np.all(alpha == alpha[0]):
                start = dict(spectral=True)
            minv = 1.0 / (beta * cn + alpha) if jacobi else None
            e = cofem_estep_pcg(op, b0, beta, alpha, K, tol, max_iter, seed, t, minv=minv, fixed_iters=fi,
                                stop_rule=stop_rule, **start)
        else:
            e = cofem_estep(op, b0, beta, alpha, K, tol, max_iter, seed, t, fi, stop_rule)
        mu, s = e.mu, e.s
        alpha_old = alpha
        alpha, n_clamped = mstep(mu, s, alpha_max)
        change = gamma_change(alpha, alpha_old)
        stats.append({"t": t, "cg_iters": e.cg.iters, "converged": e.cg.converged,
                      "rel_resid": e.cg.rel_resid, "n_clamped": n_clamped, "gamma_change": change})
        if em_tol is not None and change < em_tol:
            break
    return CoFEMResult(alpha=alpha, mu=mu, s=s, stats=stats)


# ---------------------------------------------------------------------------
# Exact EM with an explicit covariance (Eq. 3, Eq. 4) -- the reference CoFEM
# approximates; small D only.
# ---------------------------------------------------------------------------
def exact_estep(phi: np.ndarray, y: np.ndarray, beta: float, alpha: np.ndarray):
    """Sigma = (beta Phi^T Phi + diag(alpha))^{-1}, mu = beta Sigma Phi^T y (Eq. 3),
    through a Cholesky factorization.  Returns (mu, diag(Sigma), Sigma)."""
    import scipy.linalg as sla

    phi = np.asarray(phi, np.float64)
    A = beta * (phi.T @ phi) + np.diag(np.asarray(alpha, np.float64))
    c = sla.cho_factor(A, lower=True)
    mu = sla.cho_solve(c, beta * (phi.T @ np.asarray(y, np.float64)))
    Sigma = sla.cho_solve(c, np.eye(A.shape[0]))
    return mu, np.diag(Sigma).copy(), Sigma


def exact_em(phi, y, beta, T_em, alpha0=None):
    """T_em iterations of exact EM (Eq. 3 then Eq. 4) from alpha = 1."""
    D = np.asarray(phi).shape[1]
    alpha = np.ones(D) if alpha0 is None else np.asarray(alpha0, np.float64).copy()
    hist = []
    mu = dS = None
    for _ in range(T_em):
        mu, dS, _ = exact_estep(phi, y, beta, alpha)
        alpha = 1.0 / (mu * mu + dS)
        hist.append(alpha.copy())
    return alpha, mu, dS, hist


def loglik(phi, y, beta, alpha) -> float:
    """log p(y | alpha) of Eq. 2 in D-space: with A = beta Phi^T Phi + diag(alpha)
    and mu = beta A^{-1} Phi^T y,
      -1/2 [ N log 2pi - N log beta - sum log alpha + log|A|
             + beta ||y - Phi mu||^2 + sum alpha mu^2 ]
    (matrix determinant lemma and Woodbury identity applied to the marginal
    covariance C = I/beta + Phi diag(alpha)^{-1} Phi^T)."""
    import scipy.linalg as sla

    phi = np.asarray(phi, np.float64)
    y = np.asarray(y, np.float64)
    alpha = np.asarray(alpha, np.float64)
    N = phi.shape[0]
    A = beta * (phi.T @ phi) + np.diag(alpha)
    L = sla.cholesky(A, lower=True)
    logdetA = 2.0 * np.sum(np.log(np.diag(L)))
    mu = sla.cho_solve((L, True), beta * (phi.T @ y))
    r = y - phi @ mu
    quad = beta * float(r @ r) + float(np.sum(alpha * mu * mu))
    return -0.5 * (N * math.log(2 * math.pi) - N * math.log(beta)
                   - float(np.sum(np.log(alpha))) + logdetA + quad)


def loglik_direct(phi, y, beta, alpha) -> float:
    """log N(y; 0, C) with C = I/beta + Phi diag(alpha)^{-1} Phi^T formed
    explicitly (the integral of Eq. 2 done in N-space)."""
    phi = np.asarray(phi, np.float64)
    y = np.asarray(y, np.float64)
    N = phi.shape[0]
    C = np.eye(N) / beta + (phi / np.asarray(alpha, np.float64)) @ phi.T
    sign, logdet = np.linalg.slogdet(C)
    if sign <= 0:
        raise ValueError("marginal covariance not positive definite")
    return -0.5 * (N * math.log(2 * math.pi) + logdet + float(y @ np.linalg.solve(C, y)))
