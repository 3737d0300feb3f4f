"""Pins of the oracle's preconditioned CG from a starting block (the solve of
the warm-started and learned forms): identity preconditioner and zero start
reduce to the plain CG; the solution is the Cholesky one; a start at the
solution needs no iteration; a diagonal preconditioner equal to the inverse
diagonal of a diagonal A solves in one step; the stop rule is the plain one."""
import numpy as np

import oracle as O
from oracle.cofem_oracle import make_apply_A


def _problem(D=150, N=70, beta=80.0, seed=0, K=3):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((N, D)) / np.sqrt(N)
    alpha = np.exp(rng.uniform(-2.0, 6.0, D))
    B = np.concatenate([np.where(rng.random((D, K)) < 0.5, -1.0, 1.0), rng.standard_normal((D, 1)) * 10],
                       axis=1)
    return O.DenseOperator(phi), alpha, beta, beta * phi.T @ phi + np.diag(alpha), B


def test_pcg_identity_zero_start_is_plain_cg():
    op, alpha, beta, A, B = _problem()
    a = make_apply_A(op, beta, alpha)
    X1, i1 = O.pcg_solve(a, B, 1e-8, 500)
    X2, i2 = O.cg_solve(a, B, 1e-8, 500)
    assert i1.iters == i2.iters
    np.testing.assert_allclose(X1, X2, rtol=1e-9, atol=1e-12)


def test_pcg_jacobi_reaches_cholesky_solution_and_needs_fewer_steps():
    op, alpha, beta, A, B = _problem(seed=1)
    a = make_apply_A(op, beta, alpha)
    minv = 1.0 / np.diag(A)
    X, info = O.pcg_solve(a, B, 1e-10, 2000, minv=minv)
    Xe = np.linalg.solve(A, B)
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < np.linalg.cond(A) * 1e-10
    _, plain = O.cg_solve(a, B, 1e-10, 2000)
    assert info.iters < plain.iters  # alpha spans 8 decades: Jacobi pays


def test_pcg_start_at_solution_takes_no_iteration():
    op, alpha, beta, A, B = _problem(seed=2)
    a = make_apply_A(op, beta, alpha)
    Xe = np.linalg.solve(A, B)
    X, info = O.pcg_solve(a, B, 1e-8, 100, minv=np.ones(A.shape[0]), X0=Xe)
    assert info.iters == 0
    np.testing.assert_allclose(X, Xe)


def test_pcg_exact_inverse_diagonal_of_diagonal_system_one_step():
    D = 40
    rng = np.random.default_rng(3)
    d = np.exp(rng.uniform(-3, 3, D))
    B = rng.standard_normal((D, 2))
    X, info = O.pcg_solve(lambda V: d[:, None] * V if V.ndim == 2 else d * V, B, 1e-12, 50, minv=1.0 / d)
    assert info.iters == 1
    np.testing.assert_allclose(X, B / d[:, None], rtol=1e-13)


def test_pcg_stop_rule_on_unpreconditioned_residual():
    op, alpha, beta, A, B = _problem(seed=4)
    a = make_apply_A(op, beta, alpha)
    tol = 1e-6
    X, info = O.pcg_solve(a, B, tol, 1000, minv=1.0 / np.diag(A))
    h = info.history
    assert h[-1] < tol <= h[-2]
    true = O.true_relative_residual(a, X, B)
    assert true < 10 * tol


def test_estep_pcg_warm_start_layout():
    op, alpha, beta, A, B = _problem(seed=5, K=4)
    b0 = B[:, -1]
    mu0 = np.linalg.solve(A, b0)
    d0 = 1.0 / np.diag(A)
    e = O.cofem_estep_pcg(op, b0, beta, alpha, 4, 1e-9, 500, seed=3, t=2, minv=d0, mu0=mu0, d0=d0)
    ref = O.cofem_estep(op, b0, beta, alpha, 4, 1e-11, 500, seed=3, t=2)
    np.testing.assert_allclose(e.mu, ref.mu, rtol=1e-6)
    np.testing.assert_allclose(e.s, ref.s, rtol=1e-5, atol=1e-9)


def test_warm_jacobi_trajectory_equals_plain_at_tight_tolerance():
    # the E-step's solution A^-1 B does not depend on the start or the
    # preconditioner, so with solves run to 1e-12 the warm-started Jacobi
    # trajectory is the plain trajectory (same probes), while its later solves
    # need fewer iterations
    from paper_2202_12808_amd import synth
    p = synth.dense_problem(48, 128, nnz=5, beta=200.0, K=6, tol=1e-12, seed=5)
    op = O.DenseOperator(p.phi.astype(np.float64))
    r1 = O.cofem(op, p.y, p.beta, 6, p.K, tol=1e-12, max_iter=2000, seed=3)
    r2 = O.cofem(op, p.y, p.beta, 6, p.K, tol=1e-12, max_iter=2000, seed=3, warm_start=True, jacobi=True)
    assert np.allclose(r2.mu, r1.mu, rtol=1e-7, atol=1e-10 * np.abs(r1.mu).max())
    assert np.allclose(1.0 / r2.alpha, 1.0 / r1.alpha, rtol=1e-6)
    assert sum(x["cg_iters"] for x in r2.stats[1:]) < sum(x["cg_iters"] for x in r1.stats[1:])
    # jacobi alone at the first E-step with alpha = 1: a multiple of the
    # identity when the columns have equal norms is plain CG (identity check on
    # the conv dictionary, whose columns all have norm ||h||)
    q = synth.conv_problem(16, 12, 3, rho=0.05, beta=50.0, K=4, tol=1e-10, seed=2)
    cop = O.ConvOperator(q.taps.astype(np.float64), q.H, q.W)
    a = O.cofem(cop, q.y, q.beta, 1, q.K, tol=1e-10, max_iter=500, seed=1)
    b = O.cofem(cop, q.y, q.beta, 1, q.K, tol=1e-10, max_iter=500, seed=1, jacobi=True)
    assert a.stats[0]["cg_iters"] == b.stats[0]["cg_iters"]
    assert np.allclose(a.mu, b.mu, rtol=1e-9, atol=1e-12)
