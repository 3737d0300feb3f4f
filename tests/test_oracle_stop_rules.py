"""Pins of the oracle's per-column stop rule (the alternative to the joint
Frobenius test of Sec. 3.2): the columns of a multi-right-hand-side CG never
mix, so freezing a finished column must give exactly the iterate of the same
block solve in which only that column is non-zero (the joint Frobenius ratio
of such a block is that column's own ||r_c|| / ||b_c||).  The reference keeps
the block's shape so both runs do the same floating-point operations on the
column: CG amplifies a rounding-order difference exponentially once the
Krylov basis loses orthogonality, so a differently shaped run only agrees to
~1e-8 after a few dozen steps."""
import numpy as np
import pytest

import oracle as O


def _spd(D, cond, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((D, D)))
    return (Q * np.geomspace(1.0, cond, D)) @ Q.T


def _only(B, c):
    Bc = np.zeros_like(B)
    Bc[:, c] = B[:, c]
    return Bc


def test_per_column_equals_one_column_solves():
    rng = np.random.default_rng(0)
    A = _spd(200, 1e3, rng)
    apply = lambda V: A @ V  # noqa: E731
    # columns of very different size, as [p_1 .. p_K | beta Phi^T y]
    B = rng.standard_normal((200, 4)) * np.array([1.0, 1.0, 3.0, 500.0])
    tol = 1e-6
    X, info = O.cg_solve(apply, B, tol, 400, stop_rule="per_column")
    assert info.converged
    counts = []
    for c in range(B.shape[1]):
        Xc, ic = O.cg_solve(apply, _only(B, c), tol, 400)
        counts.append(ic.iters)
        assert np.array_equal(X[:, c], Xc[:, c]), c
        assert np.linalg.norm(B[:, c] - A @ X[:, c]) < 2 * tol * np.linalg.norm(B[:, c])
    assert info.iters == max(counts) and min(counts) < max(counts)


def test_per_column_zero_column_and_cap():
    rng = np.random.default_rng(1)
    A = _spd(40, 1e6, rng)
    apply = lambda V: A @ V  # noqa: E731
    B = np.concatenate([rng.standard_normal((40, 2)), np.zeros((40, 1))], axis=1)
    X, info = O.cg_solve(apply, B, 1e-12, 5, stop_rule="per_column")
    assert info.iters == 5 and not info.converged
    assert np.all(X[:, 2] == 0.0)
    for c in range(2):
        Xc, _ = O.cg_solve(apply, _only(B, c), 0.0, 5, fixed_iters=5)
        assert np.array_equal(X[:, c], Xc[:, c])
    # an all-zero block is finished before the first step
    X0, i0 = O.cg_solve(apply, np.zeros((40, 3)), 1e-6, 10, stop_rule="per_column")
    assert i0.iters == 0 and np.all(X0 == 0.0)


def test_per_column_pcg_equals_one_column_pcg():
    rng = np.random.default_rng(2)
    A = _spd(150, 1e3, rng) + np.diag(rng.uniform(1.0, 100.0, 150))
    apply = lambda V: A @ V  # noqa: E731
    B = rng.standard_normal((150, 3)) * np.array([1.0, 20.0, 0.1])
    X0 = 0.3 * rng.standard_normal((150, 3))
    minv = 1.0 / np.diag(A)
    tol = 1e-7
    X, info = O.pcg_solve(apply, B, tol, 300, minv=minv, X0=X0, stop_rule="per_column")
    assert info.converged
    for c in range(3):
        Xc, _ = O.pcg_solve(apply, _only(B, c), tol, 300, minv=minv, X0=_only(X0, c))
        assert np.array_equal(X[:, c], Xc[:, c]), c
        assert np.linalg.norm(B[:, c] - A @ X[:, c]) < 2 * tol * np.linalg.norm(B[:, c])


def test_unknown_stop_rule_rejected():
    with pytest.raises(ValueError):
        O.cg_solve(lambda V: V, np.ones((3, 1)), 1e-6, 10, stop_rule="max")
