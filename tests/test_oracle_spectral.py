"""Pins of the oracle's spectral start: with a uniform alpha = a the E-step
matrix A = beta Phi^T Phi + a I of Eq. 3 is block-circulant for a circular
convolution dictionary, and ``ConvOperatorFFT.solve_shifted`` solves it by a
division in the Fourier domain.  Checked against the direct wrap-mode stencil
(no transform involved), an explicit dense matrix and Cholesky solves, and
the exact E-step of Eq. 3 with its diagonal estimate (Eq. 6)."""
import numpy as np
import pytest

import oracle as O


def _dense_conv_matrix(op):
    """Columns of Phi as impulse responses of the direct stencil."""
    D = op.D
    return op.apply(np.eye(D))


@pytest.mark.parametrize("H,W,k", [(16, 16, 7), (8, 32, 3), (9, 13, 5), (4, 4, 3), (1, 8, 3)])
@pytest.mark.parametrize("a", [1.0, 0.37, 250.0])
def test_solve_shifted_residual_on_direct_stencil(H, W, k, a):
    # the residual of the Fourier-domain solve, evaluated with the direct
    # wrap-mode stencil (scipy.ndimage), is at rounding level
    rng = np.random.default_rng(H * 100 + W + k)
    taps = rng.standard_normal((k, k))
    taps /= np.linalg.norm(taps)
    beta = 1e3
    direct = O.ConvOperator(taps, H, W)
    fft = O.ConvOperatorFFT(taps, H, W)
    B = rng.standard_normal((H * W, 3))
    X = fft.solve_shifted(B, beta, a)
    R = B - (beta * direct.apply_t(direct.apply(X)) + a * X)
    assert np.linalg.norm(R) <= 1e-11 * np.linalg.norm(B) * (1 + beta / a)


def test_solve_shifted_equals_dense_cholesky():
    rng = np.random.default_rng(3)
    H, W, k = 6, 10, 3
    taps = rng.standard_normal((k, k))
    op = O.ConvOperator(taps, H, W)
    Phi = _dense_conv_matrix(op)
    beta, a = 40.0, 0.8
    A = beta * Phi.T @ Phi + a * np.eye(op.D)
    B = rng.standard_normal((op.D, 4))
    ref = np.linalg.solve(A, B)
    got = O.ConvOperatorFFT(taps, H, W).solve_shifted(B, beta, a)
    assert np.allclose(got, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # a single column (1-D input) too
    assert np.allclose(O.ConvOperatorFFT(taps, H, W).solve_shifted(B[:, 2], beta, a), ref[:, 2],
                       rtol=0, atol=1e-10 * np.abs(ref).max())


def test_solve_shifted_rejects_nonpositive_shift():
    op = O.ConvOperatorFFT(np.ones((3, 3)), 4, 4)
    with pytest.raises(ValueError):
        op.solve_shifted(np.ones(16), 1.0, 0.0)


def test_spectral_estep_is_the_exact_estep():
    # from the exact start the solve's own stop test holds before the first
    # iteration: mu is Eq. 3's mean and s the probe estimate (Eq. 6) of the
    # explicit covariance
    rng = np.random.default_rng(11)
    H, W, k, K = 8, 8, 5, 6
    taps = rng.standard_normal((k, k))
    taps /= np.linalg.norm(taps)
    op = O.ConvOperator(taps, H, W)
    Phi = _dense_conv_matrix(op)
    y = rng.standard_normal(op.D)
    beta = 200.0
    alpha = np.ones(op.D)
    b0 = beta * op.apply_t(y)
    e = O.cofem_estep_pcg(op, b0, beta, alpha, K, 1e-8, 50, 7, 1, spectral=True)
    assert e.cg.iters == 0
    mu, _, Sigma = O.exact_estep(Phi, y, beta, alpha)
    assert np.allclose(e.mu, mu, rtol=0, atol=1e-10 * np.abs(mu).max())
    P = O.rademacher_probes(7, 1, K, op.D)
    s_ref = np.mean(P * (Sigma @ P), axis=1)
    assert np.allclose(e.s, s_ref, rtol=0, atol=1e-12)


def test_spectral_estep_rejects_nonuniform_alpha():
    op = O.ConvOperator(np.ones((3, 3)), 4, 4)
    alpha = np.ones(16)
    alpha[3] = 2.0
    with pytest.raises(ValueError):
        O.cofem_estep_pcg(op, np.ones(16), 1.0, alpha, 2, 1e-6, 10, 1, 1, spectral=True)
    with pytest.raises(ValueError):
        O.cofem_estep_pcg(O.DenseOperator(np.eye(4)), np.ones(4), 1.0, np.ones(4), 2, 1e-6, 10, 1, 1,
                          spectral=True)


def test_cofem_spectral_start_only_while_alpha_uniform():
    # the first E-step (alpha = 1) starts exactly and stops at once; later
    # ones run their warm-started solves, and the EM fixed point is the one
    # of the plain warm-started run up to the solve tolerance
    rng = np.random.default_rng(5)
    H, W, k = 16, 16, 5
    taps = rng.standard_normal((k, k))
    taps /= np.linalg.norm(taps)
    op = O.ConvOperatorFFT(taps, H, W)
    z = np.zeros(op.D)
    z[rng.choice(op.D, 6, replace=False)] = rng.standard_normal(6)
    y = op.apply(z) + 0.01 * rng.standard_normal(op.D)
    kw = dict(K=8, tol=1e-9, max_iter=2000, seed=4, warm_start=True, jacobi=True)
    r1 = O.cofem(op, y, 1e4, 6, spectral_start=True, **kw)
    r2 = O.cofem(op, y, 1e4, 6, **kw)
    assert r1.stats[0]["cg_iters"] == 0 and r1.stats[0]["converged"]
    assert r2.stats[0]["cg_iters"] > 50
    assert all(st["cg_iters"] > 0 for st in r1.stats[1:])
    assert np.allclose(1.0 / r1.alpha, 1.0 / r2.alpha, rtol=1e-5, atol=1e-9)
    # a non-uniform alpha0 never takes the spectral start
    a0 = np.ones(op.D)
    a0[0] = 3.0
    r3 = O.cofem(op, y, 1e4, 1, alpha0=a0, spectral_start=True, **kw)
    assert r3.stats[0]["cg_iters"] > 50
