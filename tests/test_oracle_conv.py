"""Pins of the oracle's circular-convolution dictionary (a structured Phi with
a fast apply, Sec. 1 and Sec. 3.2) against the convolution theorem, adjointness
and a brute-force dense matrix."""
import numpy as np
import pytest

import oracle as O


def _fft_conv(taps, img):
    # circular convolution through the DFT: place the kernel with its centre at
    # the origin, multiply spectra
    H, W = img.shape
    kh, kw = taps.shape
    ch, cw = (kh - 1) // 2, (kw - 1) // 2
    kern = np.zeros((H, W))
    for a in range(kh):
        for b in range(kw):
            kern[(a - ch) % H, (b - cw) % W] += taps[a, b]
    return np.real(np.fft.ifft2(np.fft.fft2(kern) * np.fft.fft2(img)))


def _fft_corr(taps, img):
    H, W = img.shape
    kh, kw = taps.shape
    ch, cw = (kh - 1) // 2, (kw - 1) // 2
    kern = np.zeros((H, W))
    for a in range(kh):
        for b in range(kw):
            kern[(a - ch) % H, (b - cw) % W] += taps[a, b]
    return np.real(np.fft.ifft2(np.conj(np.fft.fft2(kern)) * np.fft.fft2(img)))


@pytest.mark.parametrize("H,W,k", [(16, 16, 7), (9, 13, 3), (32, 20, 9), (5, 5, 5)])
def test_conv_matches_fft(H, W, k):
    rng = np.random.default_rng(H * W + k)
    taps = rng.standard_normal((k, k))
    op = O.ConvOperator(taps, H, W)
    z = rng.standard_normal((H, W, 3))
    got = op.apply(z.reshape(H * W, 3)).reshape(H, W, 3)
    gt = op.apply_t(z.reshape(H * W, 3)).reshape(H, W, 3)
    for c in range(3):
        assert np.allclose(got[:, :, c], _fft_conv(taps, z[:, :, c]), atol=1e-11)
        assert np.allclose(gt[:, :, c], _fft_corr(taps, z[:, :, c]), atol=1e-11)


def test_conv_adjoint():
    rng = np.random.default_rng(1)
    op = O.ConvOperator(rng.standard_normal((7, 7)), 24, 17)
    u = rng.standard_normal(op.D)
    w = rng.standard_normal(op.D)
    assert abs(op.apply(u) @ w - u @ op.apply_t(w)) < 1e-12 * np.linalg.norm(u) * np.linalg.norm(w) * 10


def test_conv_single_pixel_response():
    # a unit impulse at (u0, v0) spreads the taps to (u0 + a - ch, v0 + b - cw)
    H, W = 11, 10
    taps = np.arange(1.0, 10.0).reshape(3, 3)
    op = O.ConvOperator(taps, H, W)
    z = np.zeros(H * W)
    u0, v0 = 0, 9
    z[u0 * W + v0] = 1.0
    out = op.apply(z).reshape(H, W)
    for a in range(3):
        for b in range(3):
            assert out[(u0 + a - 1) % H, (v0 + b - 1) % W] == taps[a, b]
    assert np.count_nonzero(out) == 9


def test_conv_cofem_equals_dense_cofem_on_its_matrix():
    # the same dictionary given as a dense matrix (columns = impulse responses)
    H, W, k = 8, 8, 3
    rng = np.random.default_rng(5)
    taps = rng.standard_normal((k, k))
    taps /= np.linalg.norm(taps)
    op = O.ConvOperator(taps, H, W)
    Phi = np.zeros((H * W, H * W))
    for j in range(H * W):
        e = np.zeros((H, W))
        e[j // W, j % W] = 1.0
        Phi[:, j] = _fft_conv(taps, e).reshape(-1)
    y = rng.standard_normal(H * W)
    r1 = O.cofem(op, y, 100.0, 4, K=5, tol=1e-12, max_iter=500, seed=9)
    r2 = O.cofem(O.DenseOperator(Phi), y, 100.0, 4, K=5, tol=1e-12, max_iter=500, seed=9)
    assert np.allclose(r1.alpha, r2.alpha, rtol=1e-7)
    assert np.allclose(r1.mu, r2.mu, rtol=1e-7, atol=1e-12)


def test_conv_column_norms():
    rng = np.random.default_rng(2)
    taps = rng.standard_normal((5, 5))
    op = O.ConvOperator(taps, 12, 12)
    e = np.zeros(op.D)
    e[37] = 1.0
    assert np.isclose(np.sum(op.apply(e) ** 2), op.column_norms_sq()[37])


@pytest.mark.parametrize("H,W,k", [(16, 16, 7), (9, 13, 3), (32, 20, 9), (5, 5, 5), (1, 8, 1)])
def test_fft_operator_matches_direct_stencil(H, W, k):
    # the convolution theorem route (ConvOperatorFFT) against the direct
    # wrap-mode stencil, for Phi, Phi^T and Phi^T Phi, one and several columns
    rng = np.random.default_rng(100 + H * W + k)
    taps = rng.standard_normal((k, k))
    direct = O.ConvOperator(taps, H, W)
    fft = O.ConvOperatorFFT(taps, H, W)
    z = rng.standard_normal((H * W, 3))
    for fn in ("apply", "apply_t"):
        ref = getattr(direct, fn)(z)
        got = getattr(fft, fn)(z)
        assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.allclose(getattr(fft, fn)(z[:, 1]), ref[:, 1], rtol=0, atol=1e-12 * np.abs(ref).max())
    g = direct.apply_t(direct.apply(z))
    assert np.allclose(fft.gram(z), g, rtol=0, atol=1e-12 * np.abs(g).max())
    assert np.allclose(fft.column_norms_sq(), direct.column_norms_sq())


def test_fft_operator_cofem_equals_direct_cofem():
    # the E-step through the fast operator follows the direct one (same probes)
    H, W, k = 24, 20, 7
    rng = np.random.default_rng(7)
    taps = rng.standard_normal((k, k))
    taps /= np.linalg.norm(taps)
    y = rng.standard_normal(H * W)
    r1 = O.cofem(O.ConvOperator(taps, H, W), y, 50.0, 3, K=6, tol=1e-11, max_iter=800, seed=3)
    r2 = O.cofem(O.ConvOperatorFFT(taps, H, W), y, 50.0, 3, K=6, tol=1e-11, max_iter=800, seed=3)
    assert np.allclose(r1.mu, r2.mu, rtol=1e-8, atol=1e-12 * np.abs(r1.mu).max())
    assert np.allclose(1.0 / r1.alpha, 1.0 / r2.alpha, rtol=1e-7)
