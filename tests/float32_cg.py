"""A float32 emulation of the GPU's CG recurrences, for the tests that bound
the float32 rounding floor of a solve (test infrastructure only).

It runs the same per-column recurrence as the library's probe columns:
float32 vectors x, r, p, q (q = A p evaluated in float32), float64 sums for
rho = r^T r, gam = p^T q, del = r^T q, eta = q^T q, and the step coefficients
a = rho / gam, b = (rho - 2 a del + a^2 eta) / rho rounded to float32 before
the updates x += a p, r -= a q, p = r + b p.  It is a model of the rounding,
not of the kernels: the GPU's stencil sums in a different order and fuses
multiply-adds, so the two float32 runs agree only to the size of the floor.
"""
import numpy as np


def conv_gram_float32(op_fft, beta, alpha):
    """q = beta Phi^T Phi p + alpha p in float32 for the oracle's
    ConvOperatorFFT (single-precision transforms)."""
    import scipy.fft as sf

    H, W = op_fft.H, op_fft.W
    spec = op_fft.gram_hat.astype(np.complex64)
    a32 = np.asarray(alpha, np.float32)
    b32 = np.float32(beta)

    def apply(V):
        img = V.reshape(H, W, -1)
        f = sf.rfft2(img, axes=(0, 1), workers=op_fft.workers)
        f *= spec[:, :, None]
        g = sf.irfft2(f, s=(H, W), axes=(0, 1), workers=op_fft.workers).reshape(H * W, -1)
        return (b32 * g.astype(np.float32) + a32[:, None] * V).astype(np.float32)

    return apply


def dense_float32(phi, beta, alpha):
    """q = beta Phi^T (Phi p) + alpha p with float32 products (single-precision
    BLAS, as the GPU's float32 MFMA passes round)."""
    ph = np.asarray(phi, np.float32)
    a32 = np.asarray(alpha, np.float32)
    b32 = np.float32(beta)

    def apply(V):
        V = np.asarray(V, np.float32)
        return (b32 * (ph.T @ (ph @ V)) + a32[:, None] * V).astype(np.float32)

    return apply


def cg_float32(apply32, B, iters, X0=None, minv=None):
    """`iters` CG steps on the float32 block B (D x n), from X0 (float32,
    R0 = B - A X0 evaluated in float32) or from zero.  With `minv` (a float32
    diagonal M^-1) the preconditioned recurrences of the library's Jacobi
    form: z = M^-1 r, rho = r^T z, del = r^T M^-1 q, eta = q^T M^-1 q, and
    p = z + b p."""
    B = np.asarray(B, np.float32)
    if X0 is None:
        X = np.zeros_like(B)
        R = B.copy()
    else:
        X = np.asarray(X0, np.float32).copy()
        R = (B - apply32(X)).astype(np.float32)
    m = None if minv is None else np.asarray(minv, np.float32)[:, None]
    Z = R.copy() if m is None else (m * R).astype(np.float32)
    P = Z.copy()
    f64 = lambda M: M.astype(np.float64)  # noqa: E731
    rho = np.einsum("dc,dc->c", f64(R), f64(Z))
    for _ in range(iters):
        Q = apply32(P)
        MQ = Q if m is None else (m * Q).astype(np.float32)
        gam = np.einsum("dc,dc->c", f64(P), f64(Q))
        dl = np.einsum("dc,dc->c", f64(R), f64(MQ))
        et = np.einsum("dc,dc->c", f64(Q), f64(MQ))
        a = np.divide(rho, gam, out=np.zeros_like(rho), where=gam != 0.0)
        rn = np.maximum(rho - 2.0 * a * dl + a * a * et, 0.0)
        b = np.divide(rn, rho, out=np.zeros_like(rho), where=rho != 0.0)
        a32, b32 = a.astype(np.float32), b.astype(np.float32)
        X = X + a32 * P
        R = R - a32 * Q
        Z = R if m is None else (m * R).astype(np.float32)
        P = Z + b32 * P
        rho = np.einsum("dc,dc->c", f64(R), f64(Z))
    return X
