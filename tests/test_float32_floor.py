"""The float32 rounding floor of the capped, ill-conditioned conv solve.

On the 256 x 256, 7x7 workload (beta = 1e4, K = 16) the first E-step's CG runs
to the cap U = 400 at kappa(A) ~ 1e5.  Float32 probe columns cannot follow the
float64 oracle's Krylov path there: a float32 model of the same recurrences
(``float32_cg``) lands 2e-4 .. 1e-3 from the oracle's diagonal estimate s.
This is the evidence behind the float32 bar of the GPU test
``test_conv_256x256_k7_fp32_error_floor`` (1e-3 on s and 1/alpha; the mean
column is float64 and still meets 1e-4), and the reason the library offers a
float64 mode for such solves.
"""
import numpy as np

import oracle as O
from paper_2202_12808_amd import synth
from tests.float32_cg import cg_float32, conv_gram_float32


def test_float32_state_floor_on_capped_conv_solve():
    p = synth.conv_256x256_k7(0)
    op = O.ConvOperatorFFT(p.taps.astype(np.float64), p.H, p.W)
    b0 = p.beta * op.apply_t(p.y.astype(np.float64))
    e = O.cofem_estep(op, b0, p.beta, np.ones(p.D), p.K, p.tol, p.max_iter, p.seed, 1,
                      fixed_iters=p.max_iter)
    assert not e.cg.converged  # capped: the regime the GPU test bounds
    P = O.rademacher_probes(p.seed, 1, p.K, p.D)
    X32 = cg_float32(conv_gram_float32(op, p.beta, np.ones(p.D)), P, p.max_iter)
    s32 = O.diag_estimate(P, X32.astype(np.float64))
    err = np.linalg.norm(s32 - e.s) / np.linalg.norm(e.s)
    print("float32-state relerr of s after the capped solve:", err)
    assert 1.5e-4 < err < 1e-3
    # the same emulation on a well-conditioned solve stays far below 1e-4:
    # the floor comes from the conditioning, not from the emulation
    alpha = np.full(p.D, 1e3)
    e2 = O.cofem_estep(op, b0, p.beta, alpha, p.K, p.tol, p.max_iter, p.seed, 1, fixed_iters=60)
    X2 = cg_float32(conv_gram_float32(op, p.beta, alpha), P, 60)
    err2 = np.linalg.norm(O.diag_estimate(P, X2.astype(np.float64)) - e2.s) / np.linalg.norm(e2.s)
    print("well-conditioned control:", err2)
    assert err2 < 1e-5
