"""CPU evidence behind two solver choices of the convolution forms, on the
oracle and on a float32 model of the GPU's CG recurrences (``float32_cg``).

1. The spectral start (the first E-step, alpha = 1): a complex-float32 DFT
   solve of the block-circulant system already lies within the solve's
   tolerance in float32 state, where zero-started float32 CG takes hundreds of
   iterations and still stops short of it.
2. The diagonal preconditioner: right after the first M-step, the diagonal of
   Sigma (what a learned diagonal would be trained towards) preconditions
   worse than the Jacobi diagonal 1 / diag(A), even taken exact.  So the
   learned form keeps Jacobi and predicts the start.
"""
import numpy as np
import scipy.fft as sf

import oracle as O
from paper_2202_12808_amd import synth
from tests.float32_cg import cg_float32, conv_gram_float32


def _problem(n=128):
    p = synth.conv_problem(n, n, 9, rho=0.01, beta=1e4, K=4, tol=1e-5, seed=1000)
    op = O.ConvOperatorFFT(p.taps.astype(np.float64), n, n)
    return p, op


def test_float32_spectral_start_meets_the_tolerance():
    p, op = _problem()
    ones = np.ones(p.D)
    A32 = conv_gram_float32(op, p.beta, ones)
    P = O.rademacher_probes(p.seed, 1, p.K, p.D).astype(np.float32)
    lam = (p.beta * op.gram_hat + 1.0).astype(np.float32)
    f = sf.rfft2(P.reshape(p.H, p.W, -1), axes=(0, 1))  # complex64 for float32 input
    assert f.dtype == np.complex64
    X0 = sf.irfft2(f / lam[:, :, None], s=(p.H, p.W), axes=(0, 1)).reshape(p.D, -1).astype(np.float32)

    def true_resid(X):  # float64 evaluation of ||P - A X|| / ||P||
        X = X.astype(np.float64)
        R = P.astype(np.float64) - (p.beta * op.gram(X) + X)
        return np.linalg.norm(R) / np.linalg.norm(P.astype(np.float64))

    # zero start: 300 float32 CG iterations stop far short of the tolerance
    rz = true_resid(cg_float32(A32, P, 300))
    r0 = true_resid(X0)
    # the model's own float32 evaluation of R0 = P - A X0 sits near the
    # tolerance, and two float32 CG iterations from X0 stay at that level
    R0 = (P - A32(X0)).astype(np.float64)
    r0_model = np.linalg.norm(R0) / np.linalg.norm(P.astype(np.float64))
    r2 = true_resid(cg_float32(A32, P, 2, X0=X0))
    print("true residual: spectral start", r0, "after 2 more", r2, "; zero start after 300:", rz,
          "; float32-model R0", r0_model)
    # (scipy's complex64 round trip leaves ~1e-5; the GPU's radix-2 start
    # measured 2e-7 at 1024^2 in float64, test_gpu_spectral.py)
    assert r0 < 2 * p.tol and r2 < 2 * p.tol
    assert r0_model < 3 * p.tol
    assert rz > 100 * r0 and rz > 10 * p.tol


def _pcg_iters(op, beta, alpha, P, X0, minv, tol=1e-5):
    B = P
    _, info = O.pcg_solve(O.make_apply_A(op, beta, alpha), B, tol, 3000, minv=minv, X0=X0)
    return info.iters


def test_jacobi_beats_diagonal_of_sigma_after_first_mstep():
    p, op = _problem(64)
    b0 = p.beta * op.apply_t(p.y.astype(np.float64))
    cn = op.column_norms_sq()
    # EM iteration 1 from alpha = 1 (exact start), its M-step, then the solve of
    # EM iteration 2 from the control's start under each diagonal
    e1 = O.cofem_estep_pcg(op, b0, p.beta, np.ones(p.D), p.K, 1e-9, 3000, p.seed, 1, spectral=True)
    alpha2, _ = O.mstep(e1.mu, e1.s)
    P = O.rademacher_probes(p.seed, 2, p.K, p.D)
    B = np.concatenate([P, b0[:, None]], axis=1)
    X0 = np.concatenate([np.maximum(e1.s, 0)[:, None] * P, e1.mu[:, None]], axis=1)
    d = p.beta * cn + alpha2
    exact = O.cofem_estep_pcg(op, b0, p.beta, alpha2, p.K, 1e-9, 3000, p.seed, 2, minv=1.0 / d)
    s2 = np.clip(exact.s, 1.0 / d, None)  # the exact next diag(Sigma) (>= 1/d_j)
    it_jac = _pcg_iters(op, p.beta, alpha2, B, X0, 1.0 / d)
    it_sig = _pcg_iters(op, p.beta, alpha2, B, X0, s2)
    it_mix = _pcg_iters(op, p.beta, alpha2, B, X0, np.sqrt(s2 / d))
    print("EM iteration 2, CG iterations: Jacobi", it_jac, "diag(Sigma)", it_sig, "sqrt(s/d)", it_mix)
    assert it_jac < it_sig and it_jac < it_mix
