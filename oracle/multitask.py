"""Plain FP64 CPU oracle of covariance-free EM for multi-task SBL.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and ``bench.py``'s
``cpu_baseline`` leg; never by the HIP product path.

The paper (Sec. 5) names multi-task SBL as an extension of CoFEM without
writing it out.  The model read here is the one of multi-task compressed
sensing with a shared prior (Ji, Dunson and Carin 2009; Wipf and Rao 2007):
T observation vectors y_t = Phi z_t + noise (precision beta), every z_t with
the same prior N(0, diag(alpha)^-1).  Given alpha the tasks are independent
and share one posterior covariance Sigma = (beta Phi^T Phi + diag(alpha))^-1;
their means are mu_t = beta Sigma Phi^T y_t.  The EM update of the shared
alpha is alpha_j = T / sum_t (mu_tj^2 + Sigma_jj).

CoFEM's E-step then solves A X = [p_1 .. p_K | beta Phi^T y_1 .. beta Phi^T y_T]
(K + T right-hand sides, probes first), reads mu_t from column K + t and
estimates diag(Sigma) from the probe columns (Eq. 6); the M-step is
alpha_j = 1 / max(mean_t mu_tj^2 + s_j, 1/alpha_max) (R6's floor).  With
T = 1 every function here reduces to the single-task one in
``cofem_oracle``.

Pins: ``tests/test_oracle_multitask.py``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .cofem_oracle import (ALPHA_MAX_DEFAULT, cg_solve, diag_estimate, exact_estep, loglik, make_apply_A,
                           rademacher_probes)


@dataclasses.dataclass
class EStepMT:
    mu: np.ndarray   # D x T
    s: np.ndarray    # D
    X: np.ndarray    # D x (K + T)
    cg: object


def cofem_estep_mt(op, B0: np.ndarray, beta: float, alpha: np.ndarray, K: int, tol: float, max_iter: int,
                   seed: int, t: int, fixed_iters: Optional[int] = None) -> EStepMT:
    """One E-step at EM iteration t: B = [P | B0] with B0 = beta Phi^T Y
    (D x T), multi-right-hand-side CG, mu_t = X[:, K + t], s from the probes."""
    D = op.D
    B0 = np.asarray(B0, np.float64).reshape(D, -1)
    P = rademacher_probes(seed, t, K, D)
    B = np.concatenate([P, B0], axis=1)
    X, info = cg_solve(make_apply_A(op, beta, alpha), B, tol, max_iter, fixed_iters)
    return EStepMT(mu=X[:, K:].copy(), s=diag_estimate(P, X[:, :K]), X=X, cg=info)


def mstep_mt(mu: np.ndarray, s: np.ndarray, alpha_max: float = ALPHA_MAX_DEFAULT):
    """alpha_j <- 1 / max(mean_t mu_tj^2 + s_j, 1/alpha_max).  Returns
    (alpha, number floored)."""
    mu = np.asarray(mu, np.float64)
    mu = mu.reshape(mu.shape[0], -1)
    denom = np.mean(mu * mu, axis=1) + np.asarray(s, np.float64)
    floor = 1.0 / alpha_max
    return 1.0 / np.maximum(denom, floor), int(np.count_nonzero(denom < floor))


@dataclasses.dataclass
class CoFEMMTResult:
    alpha: np.ndarray
    mu: np.ndarray
    s: np.ndarray
    stats: list


def cofem_mt(op, Y: np.ndarray, beta: float, T_em: int, K: int, *, tol: float, max_iter: int, seed: int,
             alpha_max: float = ALPHA_MAX_DEFAULT, alpha0: Optional[np.ndarray] = None, t0: int = 1,
             fixed_iters=None) -> CoFEMMTResult:
    """Multi-task CoFEM: T_em EM iterations from alpha = 1 (or alpha0), EM
    iterations numbered t0, t0 + 1, ... (t selects the probe draw)."""
    D = op.D
    Y = np.asarray(Y, np.float64).reshape(op.N, -1)
    alpha = np.ones(D) if alpha0 is None else np.asarray(alpha0, np.float64).copy()
    B0 = beta * op.apply_t(Y)
    stats = []
    mu = s = None
    for i in range(T_em):
        t = t0 + i
        fi = fixed_iters[i] if isinstance(fixed_iters, (list, tuple, np.ndarray)) else fixed_iters
        e = cofem_estep_mt(op, B0, beta, alpha, K, tol, max_iter, seed, t, fi)
        mu, s = e.mu, e.s
        alpha, n_clamped = mstep_mt(mu, s, alpha_max)
        stats.append({"t": t, "cg_iters": e.cg.iters, "converged": e.cg.converged, "rel_resid": e.cg.rel_resid,
                      "n_clamped": n_clamped})
    return CoFEMMTResult(alpha=alpha, mu=mu, s=s, stats=stats)


def exact_em_mt(phi, Y, beta, T_em, alpha0=None):
    """Exact multi-task EM with an explicit Sigma (small D): T_em iterations
    of mu_t = beta Sigma Phi^T y_t, alpha_j = T / sum_t (mu_tj^2 + Sigma_jj)."""
    phi = np.asarray(phi, np.float64)
    Y = np.asarray(Y, np.float64).reshape(phi.shape[0], -1)
    D = phi.shape[1]
    alpha = np.ones(D) if alpha0 is None else np.asarray(alpha0, np.float64).copy()
    mu = dS = None
    for _ in range(T_em):
        cols = [exact_estep(phi, Y[:, t], beta, alpha) for t in range(Y.shape[1])]
        mu = np.stack([c[0] for c in cols], axis=1)
        dS = cols[0][1]
        alpha = 1.0 / (np.mean(mu * mu, axis=1) + dS)
    return alpha, mu, dS


def loglik_mt(phi, Y, beta, alpha) -> float:
    """log p(Y | alpha) = sum_t log p(y_t | alpha): the tasks are independent
    given the shared alpha (Eq. 2 per task)."""
    Y = np.asarray(Y, np.float64).reshape(np.asarray(phi).shape[0], -1)
    return float(sum(loglik(phi, Y[:, t], beta, alpha) for t in range(Y.shape[1])))
