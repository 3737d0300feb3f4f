"""Pins of the multi-task oracle (shared alpha over T tasks, the extension
named in Sec. 5) against the single-task oracle, closed forms, exact
multi-task EM and its log-likelihood."""
import numpy as np

import oracle as O
from oracle import multitask as M


def _dense(N, D, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, D)) / np.sqrt(N), rng


def test_one_task_is_the_single_task_oracle():
    phi, rng = _dense(20, 40, 1)
    y = rng.standard_normal(20)
    op = O.DenseOperator(phi)
    a = M.cofem_mt(op, y[:, None], 30.0, 5, K=6, tol=1e-9, max_iter=200, seed=3)
    b = O.cofem(op, y, 30.0, 5, K=6, tol=1e-9, max_iter=200, seed=3)
    assert np.array_equal(a.alpha, b.alpha)
    assert np.array_equal(a.mu[:, 0], b.mu)
    assert np.array_equal(a.s, b.s)


def test_duplicated_tasks_give_the_single_task_alpha():
    # mean_t mu_t^2 of identical tasks is mu^2: the M-step equals the
    # single-task one (up to the joint stop's rounding)
    phi, rng = _dense(20, 40, 2)
    y = rng.standard_normal(20)
    op = O.DenseOperator(phi)
    a = M.cofem_mt(op, np.stack([y, y, y], axis=1), 30.0, 4, K=8, tol=1e-12, max_iter=400, seed=5)
    b = O.cofem(op, y, 30.0, 4, K=8, tol=1e-12, max_iter=400, seed=5)
    assert np.allclose(a.alpha, b.alpha, rtol=1e-8)
    for t in range(3):
        assert np.allclose(a.mu[:, t], b.mu, rtol=1e-8, atol=1e-12)


def test_task_order_does_not_matter():
    phi, rng = _dense(24, 48, 3)
    Y = rng.standard_normal((24, 3))
    op = O.DenseOperator(phi)
    # (the joint stop may land one iteration apart under a different summation
    # order, hence the tolerance)
    a = M.cofem_mt(op, Y, 50.0, 3, K=5, tol=1e-12, max_iter=400, seed=7)
    b = M.cofem_mt(op, Y[:, [2, 0, 1]], 50.0, 3, K=5, tol=1e-12, max_iter=400, seed=7)
    assert np.allclose(a.alpha, b.alpha, rtol=1e-8)
    assert np.allclose(a.mu[:, [2, 0, 1]], b.mu, rtol=1e-8, atol=1e-10)


def test_identity_dictionary_closed_form():
    # Phi = I: mu_tj = beta y_tj / (beta + alpha_j), Sigma_jj = 1/(beta + alpha_j),
    # alpha_j <- 1 / (mean_t mu_tj^2 + Sigma_jj), for any K (A is diagonal)
    D, T, beta = 30, 4, 20.0
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((D, T))
    r = M.cofem_mt(O.DenseOperator(np.eye(D)), Y, beta, 3, K=2, tol=1e-13, max_iter=50, seed=1)
    a = np.ones(D)
    for _ in range(3):
        mu = beta * Y / (beta + a)[:, None]
        v = 1.0 / (beta + a)
        a = 1.0 / (np.mean(mu * mu, axis=1) + v)
    assert np.allclose(r.alpha, a, rtol=1e-12)
    assert np.allclose(r.s, v, rtol=1e-12)


def test_many_probes_track_exact_multitask_em():
    phi, rng = _dense(24, 40, 5)
    Z = np.zeros((40, 3))
    Z[rng.choice(40, 5, replace=False)] = rng.standard_normal((5, 3))
    Y = phi @ Z + 0.05 * rng.standard_normal((24, 3))
    beta = 400.0
    a_x, mu_x, _ = M.exact_em_mt(phi, Y, beta, 4)
    r = M.cofem_mt(O.DenseOperator(phi), Y, beta, 4, K=4000, tol=1e-12, max_iter=400, seed=9)
    assert np.max(np.abs(np.log(r.alpha) - np.log(a_x))) < 0.1
    assert np.linalg.norm(r.mu - mu_x) < 0.02 * np.linalg.norm(mu_x)


def test_exact_multitask_em_increases_the_likelihood():
    phi, rng = _dense(16, 24, 6)
    Y = rng.standard_normal((16, 3))
    beta = 10.0
    ll = []
    alpha = np.ones(24)
    for _ in range(6):
        ll.append(M.loglik_mt(phi, Y, beta, alpha))
        alpha, _, _ = M.exact_em_mt(phi, Y, beta, 1, alpha0=alpha)
    ll.append(M.loglik_mt(phi, Y, beta, alpha))
    assert all(b >= a - 1e-9 for a, b in zip(ll, ll[1:]))
    assert ll[-1] > ll[0]


def test_mstep_floor():
    a, n = M.mstep_mt(np.zeros((4, 2)), np.array([0.0, -1.0, 1e-12, 1.0]), alpha_max=1e10)
    assert n == 3
    assert np.allclose(a, [1e10, 1e10, 1e10, 1.0])
