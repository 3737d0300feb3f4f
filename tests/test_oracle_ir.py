"""Pins of the oracle's iterative-refinement solve (the mixed-precision form).

Iterative refinement is not in the paper; the oracle follows the classical
scheme (outer residual with the problem's operator, inner CG corrections with a
lower-precision one).  Pinned here against: plain CG when the inner operator is
exact, the Cholesky solution within the tolerance, the true residual at exit,
monotone residual decrease for a contraction, and replay with fixed counts.
"""
import numpy as np
import pytest

import oracle as O
from oracle.cofem_oracle import make_apply_A, ir_solve


def _spd_problem(D=120, N=60, beta=50.0, seed=0, K=3):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((N, D)) / np.sqrt(N)
    alpha = np.exp(rng.uniform(-1.0, 2.0, D))
    B = np.concatenate([np.where(rng.random((D, K)) < 0.5, -1.0, 1.0), rng.standard_normal((D, 1)) * 30.0],
                       axis=1)
    A = beta * phi.T @ phi + np.diag(alpha)
    return phi, alpha, beta, A, B


def _bf16(x):
    # round-to-nearest-even to bfloat16 on the float32 value (test-side helper)
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_ir_with_exact_inner_operator_is_one_cg_solve():
    phi, alpha, beta, A, B = _spd_problem()
    op = O.DenseOperator(phi)
    apply_A = make_apply_A(op, beta, alpha)
    X, info = ir_solve(apply_A, apply_A, B, tol=1e-6, tol_in=1e-9, max_iter=400, max_sweeps=10)
    Xc, ci = O.cg_solve(apply_A, B, 1e-9, 400)
    assert info.sweeps == [ci.iters]
    np.testing.assert_allclose(X, Xc, rtol=0, atol=1e-12 * np.abs(Xc).max())


def test_ir_bf16_inner_reaches_true_tolerance_and_cholesky_solution():
    phi, alpha, beta, A, B = _spd_problem(seed=1)
    op, opb = O.DenseOperator(phi), O.DenseOperator(_bf16(phi))
    tol = 1e-9
    X, info = ir_solve(make_apply_A(op, beta, alpha), make_apply_A(opb, beta, alpha), B, tol=tol,
                       tol_in=1e-2, max_iter=2000, max_sweeps=50)
    assert info.converged and len(info.sweeps) >= 2
    assert O.true_relative_residual(make_apply_A(op, beta, alpha), X, B) < tol
    Xe = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < kappa * tol
    # the same run against the bf16 system instead converges to a different
    # solution: the outer residual really uses the full operator
    Xb = np.linalg.solve(beta * _bf16(phi).T @ _bf16(phi) + np.diag(alpha), B)
    assert np.linalg.norm(Xb - Xe) / np.linalg.norm(Xe) > 100 * np.linalg.norm(X - Xe) / np.linalg.norm(Xe)


def test_ir_true_residual_decreases_each_sweep_for_a_contraction():
    phi, alpha, beta, A, B = _spd_problem(seed=2)
    op, opb = O.DenseOperator(phi), O.DenseOperator(_bf16(phi))
    X, info = ir_solve(make_apply_A(op, beta, alpha), make_apply_A(opb, beta, alpha), B, tol=1e-10,
                       tol_in=1e-3, max_iter=4000, max_sweeps=40)
    h = info.history
    assert all(b < a for a, b in zip(h[:-1], h[1:]))
    assert h[-1] == pytest.approx(info.rel_resid)


def test_ir_fixed_counts_replay_a_free_run():
    phi, alpha, beta, A, B = _spd_problem(seed=3)
    op, opb = O.DenseOperator(phi), O.DenseOperator(_bf16(phi))
    a, ab = make_apply_A(op, beta, alpha), make_apply_A(opb, beta, alpha)
    X1, i1 = ir_solve(a, ab, B, tol=1e-7, tol_in=1e-2, max_iter=400, max_sweeps=10)
    X2, i2 = ir_solve(a, ab, B, tol=0.0, tol_in=0.5, max_iter=0, max_sweeps=0, fixed_inner=i1.sweeps)
    assert i2.sweeps == i1.sweeps
    np.testing.assert_array_equal(X1, X2)


def test_ir_zero_rhs_and_budget():
    phi, alpha, beta, A, B = _spd_problem(seed=4)
    op = O.DenseOperator(phi)
    a = make_apply_A(op, beta, alpha)
    X, info = ir_solve(a, a, np.zeros_like(B), tol=1e-6, tol_in=1e-2, max_iter=100, max_sweeps=5)
    assert info.sweeps == [] and not X.any()
    X, info = ir_solve(a, a, B, tol=1e-30, tol_in=1e-1, max_iter=7, max_sweeps=100)
    assert info.iters <= 7 and not info.converged


def test_estep_ir_matches_plain_estep_when_inner_is_exact():
    phi, alpha, beta, A, B = _spd_problem(seed=5, K=4)
    op = O.DenseOperator(phi)
    b0 = B[:, -1]
    e_ir, info = O.cofem_estep_ir(op, op, b0, beta, alpha, 4, 1e-8, 1e-12, 400, 10, seed=9, t=2)
    e = O.cofem_estep(op, b0, beta, alpha, 4, 1e-12, 400, seed=9, t=2)
    assert len(info.sweeps) == 1
    np.testing.assert_allclose(e_ir.mu, e.mu, rtol=1e-12, atol=0)
    np.testing.assert_allclose(e_ir.s, e.s, rtol=1e-12, atol=1e-15)


def test_ir_stops_after_three_stalled_sweeps():
    # an inner operator so far from A that refinement cannot contract (A/5:
    # every correction overshoots, R -> -4 R): the loop ends after IR_STALL
    # sweeps without halving the best ratio
    phi, alpha, beta, A, B = _spd_problem(seed=6)
    op = O.DenseOperator(phi)
    a = make_apply_A(op, beta, alpha)
    bad = make_apply_A(op, 0.2 * beta, 0.2 * alpha)
    X, info = ir_solve(a, bad, B, tol=1e-12, tol_in=1e-6, max_iter=10000, max_sweeps=100)
    h = info.history
    assert not info.converged and len(info.sweeps) < 100
    best = h[0]
    stall = 0
    for r in h[1:]:
        if r < 0.5 * best:
            best, stall = r, 0
        else:
            stall += 1
    assert stall == 3 and len(info.sweeps) == 3


def test_ir_warm_start_pins():
    # X0 = 0 is the cold start; X0 = the exact solution needs no sweep; any
    # other X0 converges to the same solution (the refinement corrects X0)
    rng = np.random.default_rng(21)
    N, D = 30, 50
    phi = rng.standard_normal((N, D)) / np.sqrt(N)
    alpha = rng.uniform(0.5, 4.0, D)
    A = lambda X: 20.0 * phi.T @ (phi @ X) + alpha[:, None] * X
    B = rng.standard_normal((D, 3))
    X_ex = np.linalg.solve(20.0 * phi.T @ phi + np.diag(alpha), B)
    cold, ic = O.ir_solve(A, A, B, 1e-10, 1e-2, 400, 20)
    zero, iz = O.ir_solve(A, A, B, 1e-10, 1e-2, 400, 20, X0=np.zeros_like(B))
    assert np.array_equal(cold, zero) and ic.sweeps == iz.sweeps
    ex, ie = O.ir_solve(A, A, B, 1e-10, 1e-2, 400, 20, X0=X_ex)
    assert ie.sweeps == [] and np.array_equal(ex, X_ex)
    X0 = X_ex * (1.0 + 1e-3 * rng.standard_normal(B.shape))
    w, iw = O.ir_solve(A, A, B, 1e-10, 1e-2, 400, 20, X0=X0)
    assert iw.converged and np.allclose(w, X_ex, rtol=1e-8, atol=1e-10)
    # a start near the solution saves sweeps against the cold start
    assert len(iw.sweeps) < len(ic.sweeps)


def test_estep_ir_warm_start_matches_pcg_warm_start():
    # the same X0 = [d0 (.) p_k | mu0] in the refinement and in PCG; with the
    # problem's own Phi as the inner operator both solve to the same X
    rng = np.random.default_rng(22)
    N, D, K = 24, 40, 4
    phi = rng.standard_normal((N, D)) / np.sqrt(N)
    op = O.DenseOperator(phi)
    y = rng.standard_normal(N)
    alpha = rng.uniform(0.5, 4.0, D)
    b0 = 10.0 * op.apply_t(y)
    mu0 = rng.standard_normal(D)
    d0 = rng.uniform(0.0, 0.2, D)
    e_ir, info = O.cofem_estep_ir(op, op, b0, 10.0, alpha, K, 1e-11, 1e-3, 400, 20, seed=5, t=3, mu0=mu0, d0=d0)
    e_pcg = O.cofem_estep_pcg(op, b0, 10.0, alpha, K, 1e-11, 400, seed=5, t=3, mu0=mu0, d0=d0)
    assert info.converged
    assert np.allclose(e_ir.X, e_pcg.X, rtol=1e-8, atol=1e-10)



def test_ir_with_jacobi_inner_solves():
    # the preconditioned inner solves: with the exact inner operator one sweep
    # is one PCG solve from zero; with the bf16 inner operator the refinement
    # reaches the true tolerance and the Cholesky solution, in fewer inner
    # iterations than the unpreconditioned refinement on this badly scaled
    # diagonal (alpha spread over three orders of magnitude)
    phi, alpha, beta, A, B = _spd_problem(seed=3)
    alpha = np.exp(np.random.default_rng(4).uniform(-2.0, 5.0, alpha.size))
    A = beta * phi.T @ phi + np.diag(alpha)
    op, opb = O.DenseOperator(phi), O.DenseOperator(_bf16(phi))
    minv = 1.0 / (beta * op.column_norms_sq() + alpha)
    apply_A = make_apply_A(op, beta, alpha)
    X, info = ir_solve(apply_A, apply_A, B, tol=1e-6, tol_in=1e-9, max_iter=400, max_sweeps=10, minv=minv)
    Xp, pi = O.pcg_solve(apply_A, B, 1e-9, 400, minv=minv)
    assert info.sweeps == [pi.iters]
    np.testing.assert_allclose(X, Xp, rtol=0, atol=1e-12 * np.abs(Xp).max())
    tol = 1e-9
    Xj, ij = ir_solve(apply_A, make_apply_A(opb, beta, alpha), B, tol=tol, tol_in=1e-2, max_iter=4000,
                      max_sweeps=50, minv=minv)
    Xn, inn = ir_solve(apply_A, make_apply_A(opb, beta, alpha), B, tol=tol, tol_in=1e-2, max_iter=4000,
                       max_sweeps=50)
    assert ij.converged and O.true_relative_residual(apply_A, Xj, B) < tol
    Xe = np.linalg.solve(A, B)
    assert np.linalg.norm(Xj - Xe) / np.linalg.norm(Xe) < np.linalg.cond(A) * tol
    print("inner iterations with and without Jacobi:", ij.iters, inn.iters)
    assert ij.iters < inn.iters


def test_estep_ir_jacobi_matches_pcg():
    # E-step with the refinement's preconditioned inner solves and the
    # problem's own Phi inside: the preconditioned E-step's X
    rng = np.random.default_rng(23)
    N, D, K = 24, 40, 4
    phi = rng.standard_normal((N, D)) / np.sqrt(N)
    op = O.DenseOperator(phi)
    y = rng.standard_normal(N)
    alpha = rng.uniform(0.5, 40.0, D)
    b0 = 10.0 * op.apply_t(y)
    minv = 1.0 / (10.0 * op.column_norms_sq() + alpha)
    e_ir, info = O.cofem_estep_ir(op, op, b0, 10.0, alpha, K, 1e-11, 1e-3, 400, 20, seed=5, t=3, minv=minv)
    e_pcg = O.cofem_estep_pcg(op, b0, 10.0, alpha, K, 1e-11, 400, seed=5, t=3, minv=minv)
    assert info.converged
    assert np.allclose(e_ir.X, e_pcg.X, rtol=1e-8, atol=1e-10)
