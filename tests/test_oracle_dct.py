"""Pins of the oracle's DCT dictionary (inverse DCT followed by an undersampling
mask, Sec. 4 "Structured Dictionary") against a brute-force cosine matrix,
orthonormality, the transform of a constant, and CoFEM run on the same
dictionary given densely."""
import math

import numpy as np
import pytest

import oracle as O


def _cosine_matrix(D):
    # orthonormal DCT-II written out element by element
    C = np.zeros((D, D))
    for k in range(D):
        ck = math.sqrt((1.0 if k == 0 else 2.0) / D)
        for n in range(D):
            C[k, n] = ck * math.cos(math.pi * (2 * n + 1) * k / (2 * D))
    return C


def _rows(D, N, seed):
    return np.sort(np.random.default_rng(seed).choice(D, N, replace=False))


@pytest.mark.parametrize("D,N", [(16, 4), (16, 16), (24, 7)])
def test_dct_matches_cosine_matrix(D, N):
    rows = _rows(D, N, 3)
    op = O.DctMaskOperator(rows, D)
    Phi = _cosine_matrix(D).T[rows]
    rng = np.random.default_rng(4)
    V = rng.standard_normal((D, 3))
    W = rng.standard_normal((N, 3))
    assert np.allclose(op.apply(V), Phi @ V, atol=1e-13)
    assert np.allclose(op.apply_t(W), Phi.T @ W, atol=1e-13)
    assert np.allclose(op.apply(V[:, 0]), Phi @ V[:, 0], atol=1e-13)


def test_dct_rows_are_orthonormal():
    D, N = 64, 16
    op = O.DctMaskOperator(_rows(D, N, 5), D)
    # Phi Phi^T = I_N, and Phi^T Phi is a projection of trace N
    G = op.apply(op.apply_t(np.eye(N)))
    assert np.allclose(G, np.eye(N), atol=1e-13)
    Pm = op.apply_t(op.apply(np.eye(D)))
    assert np.allclose(Pm @ Pm, Pm, atol=1e-13)
    assert math.isclose(np.trace(Pm), N, rel_tol=1e-12)


def test_dct_of_a_constant_signal():
    # with every sample observed Phi = C^T: a constant signal has only the
    # zero-frequency coefficient, sqrt(D) times the constant
    D = 32
    op = O.DctMaskOperator(np.arange(D), D)
    z = op.apply_t(np.full(D, 2.0))
    assert math.isclose(z[0], 2.0 * math.sqrt(D), rel_tol=1e-13)
    assert np.abs(z[1:]).max() < 1e-13
    # and the two-point transform is the normalised sum and difference
    op2 = O.DctMaskOperator(np.arange(2), 2)
    assert np.allclose(op2.apply_t(np.array([3.0, 1.0])), [4.0 / math.sqrt(2), 2.0 / math.sqrt(2)])


def test_dct_column_norms():
    D, N = 24, 9
    rows = _rows(D, N, 6)
    op = O.DctMaskOperator(rows, D)
    Phi = _cosine_matrix(D).T[rows]
    assert np.allclose(op.column_norms_sq(), np.sum(Phi * Phi, axis=0), atol=1e-13)
    assert math.isclose(op.column_norms_sq().sum(), N, rel_tol=1e-12)


def test_dct_rejects_bad_rows():
    with pytest.raises(ValueError):
        O.DctMaskOperator(np.array([0, 3, 3]), 8)
    with pytest.raises(ValueError):
        O.DctMaskOperator(np.array([0, 8]), 8)


def test_dct_cofem_equals_dense_cofem_on_its_matrix():
    D, N = 32, 8
    rows = _rows(D, N, 7)
    Phi = _cosine_matrix(D).T[rows]
    rng = np.random.default_rng(8)
    y = rng.standard_normal(N)
    r1 = O.cofem(O.DctMaskOperator(rows, D), y, 50.0, 4, K=6, tol=1e-12, max_iter=500, seed=11)
    r2 = O.cofem(O.DenseOperator(Phi), y, 50.0, 4, K=6, tol=1e-12, max_iter=500, seed=11)
    assert np.allclose(r1.alpha, r2.alpha, rtol=1e-7)
    assert np.allclose(r1.mu, r2.mu, rtol=1e-7, atol=1e-12)


def test_dct_cofem_approaches_exact_em():
    # with many probes and a tight tolerance the E-step's diagonal estimate is
    # close to the exact posterior variances (Eq. 6 against Eq. 3)
    D, N = 32, 12
    rows = _rows(D, N, 9)
    Phi = _cosine_matrix(D).T[rows]
    rng = np.random.default_rng(10)
    alpha = rng.uniform(0.5, 5.0, D)
    y = rng.standard_normal(N)
    beta = 20.0
    op = O.DctMaskOperator(rows, D)
    e = O.cofem_estep(op, beta * op.apply_t(y), beta, alpha, 4000, 1e-12, 500, 12, 1)
    mu_x, sig_x, _ = O.exact_estep(Phi, y, beta, alpha)
    assert np.allclose(e.mu, mu_x, rtol=1e-8, atol=1e-10)
    assert np.abs(e.s - sig_x).max() < 0.05 * np.abs(sig_x).max()
