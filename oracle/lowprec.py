"""Low-precision dictionaries and the contraction of iterative refinement
(float64 CPU oracle; TEST INFRASTRUCTURE ONLY: used by ``tests/``, never by
the HIP product path).

Not in the paper: the mixed-precision form of the E-step solves A X = B
(A = beta Phi^T Phi + diag(alpha), Eq. 7) by iterative refinement whose inner
solves use A~ = beta Phi~^T Phi~ + diag(alpha) with a rounded dictionary
Phi~.  With exact inner solves the error obeys e' = (I - A~^-1 A) e, so the
refinement converges iff the spectral radius of I - A~^-1 A is below one.

* ``round_to_e4m3``: OCP 8-bit floating point E4M3 (1 sign bit, 4 exponent
  bits with bias 7, 3 mantissa bits; subnormals below 2^-6 in steps of 2^-9;
  largest finite 448; no infinities), round to nearest, ties to even,
  saturating at +-448.
* ``e4m3_dictionary``: Phi scaled by one power of two (the largest 2^e with
  max |Phi| 2^e <= 448), rounded to E4M3, scaled back (exact).
* ``refinement_contraction``: max |1 - lambda| over the eigenvalues lambda of
  A~^-1 A (computed as the symmetric L^-1 A L^-T, A~ = L L^T).
* ``conv_refinement_contraction``: the same for a circular-convolution
  dictionary under a uniform alpha = a, where A and A~ share the 2D DFT as
  eigenvectors: lambda_k = (beta |h_hat_k|^2 + a) / (beta |h~_hat_k|^2 + a).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def round_to_e4m3(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    # exponent of the binade (normal numbers 2^-6 .. 2^8); the subnormal range
    # below 2^-6 has the spacing of the 2^-6 binade, 2^-9
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.clip(e, -6, 8)
    step = np.ldexp(1.0, (e - 3).astype(np.int64))
    q = np.round(a / step) * step  # numpy rounds half to even
    q = np.minimum(q, E4M3_MAX)
    return np.where(a > 0, np.copysign(q, x), 0.0 * x)


def decode_e4m3(code: int) -> float:
    """Value of the 8-bit E4M3 code (bit 7 sign, bits 6..3 exponent, 2..0
    mantissa); None for the NaN codes 0x7F and 0xFF."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return None
    if e == 0:
        return s * m * 2.0 ** -9
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def e4m3_dictionary(phi: np.ndarray):
    """(Phi~, scale): Phi~ = round_to_e4m3(Phi * scale) / scale with scale the
    largest power of two that keeps max |Phi| scale <= 448."""
    phi = np.asarray(phi, np.float64)
    m = float(np.abs(phi).max())
    scale = 2.0 ** np.floor(np.log2(E4M3_MAX / m)) if m > 0 else 1.0
    return round_to_e4m3(phi * scale) / scale, scale


def refinement_contraction(phi: np.ndarray, phi_low: np.ndarray, beta: float, alpha: np.ndarray) -> float:
    """Spectral radius of I - A~^-1 A for A = beta Phi^T Phi + diag(alpha) and
    A~ the same with phi_low (dense eigen-decomposition: small D only)."""
    phi = np.asarray(phi, np.float64)
    phi_low = np.asarray(phi_low, np.float64)
    alpha = np.asarray(alpha, np.float64)
    A = beta * (phi.T @ phi) + np.diag(alpha)
    At = beta * (phi_low.T @ phi_low) + np.diag(alpha)
    L = np.linalg.cholesky(At)
    Li = np.linalg.solve(L, np.eye(L.shape[0]))
    ev = np.linalg.eigvalsh(Li @ A @ Li.T)
    return float(max(abs(1.0 - ev.min()), abs(1.0 - ev.max())))


def conv_refinement_contraction(taps: np.ndarray, taps_low: np.ndarray, H: int, W: int, beta: float,
                                a: float) -> float:
    """Spectral radius of I - A~^-1 A for the circular convolution with
    `taps` (A) and with `taps_low` (A~) on an H x W image, alpha = a
    everywhere: max_k |beta (g~_k - g_k)| / (beta g~_k + a) with g = |h_hat|^2
    from the oracle's Fourier-domain operator (any image size)."""
    from .cofem_oracle import ConvOperatorFFT

    g = ConvOperatorFFT(np.asarray(taps, np.float64), H, W).gram_hat
    gl = ConvOperatorFFT(np.asarray(taps_low, np.float64), H, W).gram_hat
    return float(np.max(np.abs(beta * (gl - g)) / (beta * gl + a)))
