"""Seeded synthetic sparse-coding problems (the compressed-sensing simulation of
Sec. 4): a dictionary Phi, a sparse ground truth z*, and y = Phi z* + noise.

This module only draws inputs.  It holds none of CoFEM's arithmetic; both the
HIP path's tests and the FP64 oracle take their inputs from here.

Recipes (one per named workload; the generative model is Eq. 1 with the noise
precision beta known):

* ``dense_256x1024``    Phi 256x1024 iid N(0, 1/N); 20 nonzeros at uniform
                        positions, N(0,1) values; beta = 1e4; K = 20; eps 1e-6;
                        U = 400; T_em = 50.
* ``dense_4096x16384``  Phi 4096x16384 iid N(0, 1/N); 1% nonzeros N(0,1);
                        beta = 1e3; K = 32; eps 1e-5; U = 400; T_em = 30.
* ``conv_256x256_k7``   2D circular convolution, 7x7 taps iid N(0,1) scaled to
                        unit l2 norm, 256x256 image; 2% nonzeros Laplace(1);
                        beta = 1e4; K = 16; eps 1e-5; U = 400; T_em = 30.
* ``conv_1024x1024_k9`` same law, 9x9 taps, 1024x1024 image; 1% nonzeros
                        N(0,1); beta = 1e4; K = 16; eps 1e-5; U = 400; T_em = 30.
* ``dct_4096``          inverse DCT (orthonormal DCT-III) of length D = 4096
                        followed by N = D/4 samples uniform without replacement;
                        4% nonzero N(0,1) coefficients; beta = 4e4 (noise sigma
                        0.005, the paper's dense setting; the DCT runs state
                        none); K = 20; eps 1e-5; U = 400; T_em = 30.
* ``dct_262144``        the same law at D = 2^18 with 10% nonzeros and T_em = 50
                        (the high-dimensional DCT runs of Sec. 4; about 50 EM
                        iterations reach their 2% NRMSE target).
* ``dct_multitask``     T tasks on one DCT dictionary (the multi-task extension
                        named in Sec. 5): a shared support of round(rho D)
                        positions, independent N(0,1) values per task.
* ``batched_64``        64 dense problems, D_i = 4*U{256..4096}, N_i = D_i/4,
                        Phi iid N(0, 1/N_i) rounded to bfloat16; 2% nonzeros
                        N(0,1); beta = 1e3; K = 16; eps 1e-5; U = 400; T_em = 30.

The number of nonzeros is round(rho * D) (half up), positions uniform without
replacement.  Phi and y are stored in float32 (the stored values are the
problem); z* stays float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    kind: str                      # "dense" | "conv" | "dct"
    N: int
    D: int
    y: np.ndarray                  # float32 (N,)
    z: np.ndarray                  # float64 (D,) ground truth
    beta: float
    K: int
    tol: float
    max_iter: int
    T_em: int
    seed: int
    phi: Optional[np.ndarray] = None    # float32 (N, D), row-major
    taps: Optional[np.ndarray] = None   # float32 (kh, kw)
    rows: Optional[np.ndarray] = None   # int32 (N,) observed samples (DCT dictionary)
    tasks: int = 1                      # T > 1: y is (T, N) and z is (T, D) (multi-task)
    H: int = 0
    W: int = 0
    name: str = ""


def _sparse_signal(rng, D, nnz, law):
    z = np.zeros(D)
    pos = rng.choice(D, size=nnz, replace=False)
    if law == "normal":
        z[pos] = rng.standard_normal(nnz)
    elif law == "laplace":
        z[pos] = rng.laplace(0.0, 1.0, nnz)
    elif law == "spikes":
        z[pos] = rng.choice(np.array([-1.0, 1.0]), size=nnz)
    else:
        raise ValueError(law)
    return z


def _nnz(rho, D):
    return int(math.floor(rho * D + 0.5))


def dense_problem(N, D, *, nnz=None, rho=None, beta, K, tol, max_iter=400, T_em=30,
                  seed=0, law="normal", bf16=False, name="") -> Problem:
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((N, D), dtype=np.float32)
    phi *= np.float32(1.0 / math.sqrt(N))
    if bf16:
        phi = round_to_bf16(phi)
    if nnz is None:
        nnz = _nnz(rho, D)
    z = _sparse_signal(rng, D, nnz, law)
    noise = rng.standard_normal(N) / math.sqrt(beta)
    y = (phi.astype(np.float64) @ z + noise).astype(np.float32)
    return Problem("dense", N, D, y, z, float(beta), K, tol, max_iter, T_em, seed,
                   phi=phi, name=name)


def conv_taps(rng, kh, kw):
    h = rng.standard_normal((kh, kw))
    h /= np.linalg.norm(h)
    return h.astype(np.float32)


def _circ_conv_f64(taps, img):
    """Forward model for data synthesis only (direct circular convolution)."""
    kh, kw = taps.shape
    ch, cw = (kh - 1) // 2, (kw - 1) // 2
    out = np.zeros_like(img)
    for a in range(kh):
        for b in range(kw):
            out += float(taps[a, b]) * np.roll(img, (a - ch, b - cw), axis=(0, 1))
    return out


def conv_problem(H, W, k, *, rho, beta, K, tol, max_iter=400, T_em=30, seed=0,
                 law="normal", name="") -> Problem:
    rng = np.random.default_rng(seed)
    taps = conv_taps(rng, k, k)
    D = H * W
    z = _sparse_signal(rng, D, _nnz(rho, D), law)
    clean = _circ_conv_f64(taps.astype(np.float64), z.reshape(H, W)).reshape(D)
    y = (clean + rng.standard_normal(D) / math.sqrt(beta)).astype(np.float32)
    return Problem("conv", D, D, y, z, float(beta), K, tol, max_iter, T_em, seed,
                   taps=taps, H=H, W=W, name=name)


def conv_multitask(H, W, k, T, *, rho, beta, K, tol, max_iter=400, T_em=30, seed=0, name="") -> Problem:
    """T tasks on one circular-convolution dictionary (taps as conv_problem):
    the signals share their support (round(rho D) pixels, uniform) with
    independent N(0,1) values per task; y_t = Phi z_t + N(0, 1/beta) noise."""
    rng = np.random.default_rng(seed)
    taps = conv_taps(rng, k, k)
    D = H * W
    pos = rng.choice(D, size=_nnz(rho, D), replace=False)
    Z = np.zeros((T, D))
    Z[:, pos] = rng.standard_normal((T, len(pos)))
    Y = np.stack([_circ_conv_f64(taps.astype(np.float64), Z[t].reshape(H, W)).reshape(D) for t in range(T)])
    Y = (Y + rng.standard_normal((T, D)) / math.sqrt(beta)).astype(np.float32)
    return Problem("conv", D, D, Y, Z, float(beta), K, tol, max_iter, T_em, seed, taps=taps, H=H, W=W,
                   tasks=T, name=name)


def dense_multitask(N, D, T, *, rho, beta, K, tol, max_iter=400, T_em=30, seed=0, name="") -> Problem:
    """T tasks on one dense dictionary (iid N(0, 1/N) as dense_problem) with a
    shared support and independent N(0,1) values per task."""
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((N, D), dtype=np.float32)
    phi *= np.float32(1.0 / math.sqrt(N))
    pos = rng.choice(D, size=_nnz(rho, D), replace=False)
    Z = np.zeros((T, D))
    Z[:, pos] = rng.standard_normal((T, len(pos)))
    Y = (Z @ phi.astype(np.float64).T + rng.standard_normal((T, N)) / math.sqrt(beta)).astype(np.float32)
    return Problem("dense", N, D, Y, Z, float(beta), K, tol, max_iter, T_em, seed, phi=phi, tasks=T, name=name)


def _inverse_dct_f64(z):
    """Forward model for data synthesis only: the orthonormal inverse DCT
    (scipy's DCT-III) of the coefficient vector."""
    import scipy.fft as sf

    return sf.idct(np.asarray(z, np.float64), type=2, norm="ortho")


def dct_problem(D, *, rho, beta, K, tol, max_iter=400, T_em=30, seed=0, name="") -> Problem:
    """Phi = inverse DCT followed by the selection of N = D/4 samples drawn
    uniformly without replacement (sorted); z* has round(rho D) N(0,1)
    coefficients; y = Phi z* + N(0, 1/beta) noise."""
    rng = np.random.default_rng(seed)
    N = D // 4
    rows = np.sort(rng.choice(D, size=N, replace=False)).astype(np.int32)
    z = _sparse_signal(rng, D, _nnz(rho, D), "normal")
    clean = _inverse_dct_f64(z)[rows]
    y = (clean + rng.standard_normal(N) / math.sqrt(beta)).astype(np.float32)
    return Problem("dct", N, D, y, z, float(beta), K, tol, max_iter, T_em, seed, rows=rows, name=name)


def dct_multitask(D, T, *, rho, beta, K, tol, max_iter=400, T_em=30, seed=0, name="") -> Problem:
    """T tasks on one DCT dictionary (N = D/4 samples as in dct_problem): the
    signals share their support (round(rho D) positions, uniform) with
    independent N(0,1) values per task; y_t = Phi z_t + N(0, 1/beta) noise."""
    rng = np.random.default_rng(seed)
    N = D // 4
    rows = np.sort(rng.choice(D, size=N, replace=False)).astype(np.int32)
    nnz = _nnz(rho, D)
    pos = rng.choice(D, size=nnz, replace=False)
    Z = np.zeros((T, D))
    Z[:, pos] = rng.standard_normal((T, nnz))
    Y = np.stack([_inverse_dct_f64(Z[t])[rows] for t in range(T)])
    Y = (Y + rng.standard_normal((T, N)) / math.sqrt(beta)).astype(np.float32)
    return Problem("dct", N, D, Y, Z, float(beta), K, tol, max_iter, T_em, seed, rows=rows, tasks=T, name=name)


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


# ---- the named workloads -------------------------------------------------
def dense_256x1024(seed=0):
    return dense_problem(256, 1024, nnz=20, beta=1e4, K=20, tol=1e-6, max_iter=400,
                         T_em=50, seed=seed, name="dense_256x1024")


def dense_4096x16384(seed=0):
    return dense_problem(4096, 16384, rho=0.01, beta=1e3, K=32, tol=1e-5, max_iter=400,
                         T_em=30, seed=seed, name="dense_4096x16384")


def conv_256x256_k7(seed=0):
    return conv_problem(256, 256, 7, rho=0.02, beta=1e4, K=16, tol=1e-5, max_iter=400,
                        T_em=30, seed=seed, law="laplace", name="conv_256x256_k7")


def conv_1024x1024_k9(seed=0):
    return conv_problem(1024, 1024, 9, rho=0.01, beta=1e4, K=16, tol=1e-5, max_iter=400,
                        T_em=30, seed=seed, law="normal", name="conv_1024x1024_k9")


def dct_4096(seed=0):
    return dct_problem(4096, rho=0.04, beta=4e4, K=20, tol=1e-5, max_iter=400, T_em=30, seed=seed,
                       name="dct_4096")


def dct_262144(seed=0):
    return dct_problem(262144, rho=0.1, beta=4e4, K=20, tol=1e-5, max_iter=400, T_em=50, seed=seed,
                       name="dct_262144")


def batched_sizes(seed=0, count=64):
    rng = np.random.default_rng(10_000 + seed)
    return [4 * int(v) for v in rng.integers(256, 4097, size=count)]


def batched_64(seed=0, count=64, sizes=None):
    sizes = batched_sizes(seed, count) if sizes is None else sizes
    return [dense_problem(D // 4, D, rho=0.02, beta=1e3, K=16, tol=1e-5, max_iter=400,
                          T_em=30, seed=seed * 1000 + i, bf16=True, name=f"batched_{i}")
            for i, D in enumerate(sizes)]


WORKLOADS = {
    "dense_256x1024": dense_256x1024,
    "dense_4096x16384": dense_4096x16384,
    "conv_256x256_k7": conv_256x256_k7,
    "conv_1024x1024_k9": conv_1024x1024_k9,
    "dct_4096": dct_4096,
    "dct_262144": dct_262144,
}
