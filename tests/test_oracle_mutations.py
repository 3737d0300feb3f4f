"""Plants plausible mistakes in the oracle (on the CPU only) and checks that at
least one pin catches each: a dropped beta, a sign error in CG, a wrong divisor
in the diagonal estimate, a transposed convolution, an off-by-one probe bit, an
M-step without s and the mean read from the wrong column."""
import numpy as np
import pytest

import oracle
import oracle.cofem_oracle as OC
from tests import test_oracle_conv as TC
from tests import test_oracle_pins as TP
from tests import test_oracle_rng as TR


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(OC, name, fn)
    if hasattr(oracle, name):
        monkeypatch.setattr(oracle, name, fn)


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_dropped_beta_is_caught(monkeypatch):
    def make_apply_A(op, beta, alpha):
        alpha = np.asarray(alpha, np.float64)
        return lambda V: op.apply_t(op.apply(V)) + (alpha[:, None] * V if V.ndim == 2 else alpha * V)
    _patch(monkeypatch, "make_apply_A", make_apply_A)
    _fails(TP.test_identity_dictionary_closed_form, "dense")


def test_cg_sign_error_is_caught(monkeypatch):
    # residual updated with the wrong sign (r += a q)
    def cg_bad(apply_A, B, tol, max_iter, fixed_iters=None):
        X = np.zeros_like(B)
        R = B.copy()
        P = R.copy()
        rho = np.einsum("dc,dc->c", R, R)
        for it in range(fixed_iters if fixed_iters is not None else max_iter):
            Q = apply_A(P)
            a = rho / np.einsum("dc,dc->c", P, Q)
            X += a * P
            R += a * Q
            rho_new = np.einsum("dc,dc->c", R, R)
            P = R + (rho_new / rho) * P
            rho = rho_new
        return X, OC.CGInfo(it + 1, True, 0.0, [])
    _patch(monkeypatch, "cg_solve", cg_bad)
    _fails(TP.test_cg_matches_cholesky_solve)


def test_cg_direction_update_error_is_caught(monkeypatch):
    # steepest descent instead of CG (direction update dropped)
    def sd(apply_A, B, tol, max_iter, fixed_iters=None):
        X = np.zeros_like(B)
        R = B.copy()
        n = fixed_iters if fixed_iters is not None else max_iter
        for it in range(n):
            Q = apply_A(R)
            a = np.einsum("dc,dc->c", R, R) / np.einsum("dc,dc->c", R, Q)
            X += a * R
            R -= a * Q
        return X, OC.CGInfo(n, True, 0.0, [])
    _patch(monkeypatch, "cg_solve", sd)
    _fails(TP.test_cg_finite_termination_on_three_eigenvalues)


def test_diag_divisor_error_is_caught(monkeypatch):
    _patch(monkeypatch, "diag_estimate", lambda P, X: np.sum(P * X, axis=1) / (P.shape[1] + 1))
    _fails(TP.test_diag_estimate_brute_force_all_sign_vectors)


def test_transposed_convolution_is_caught(monkeypatch):
    monkeypatch.setattr(OC.ConvOperator, "apply", OC.ConvOperator.apply_t)
    _fails(TC.test_conv_matches_fft, 16, 16, 7)


def test_probe_bit_off_by_one_is_caught(monkeypatch, golden_dir):
    orig = OC.rademacher_probes

    def shifted(seed, t, K, D):
        P = orig(seed, t, K, D + 1)
        return P[1:]
    _patch(monkeypatch, "rademacher_probes", shifted)
    _fails(TR.test_probe_bits_follow_stream_words, golden_dir)


def test_mstep_without_s_is_caught(monkeypatch):
    def mstep(mu, s, alpha_max=OC.ALPHA_MAX_DEFAULT):
        return 1.0 / np.maximum(mu * mu, 1.0 / alpha_max), 0
    _patch(monkeypatch, "mstep", mstep)
    _fails(TP.test_identity_dictionary_closed_form, "conv")


def test_mean_from_wrong_column_is_caught(monkeypatch):
    orig = OC.cofem_estep

    def bad(op, b0, beta, alpha, K, tol, max_iter, seed, t, fixed_iters=None, stop_rule="frobenius"):
        e = orig(op, b0, beta, alpha, K, tol, max_iter, seed, t, fixed_iters, stop_rule)
        e.mu = e.X[:, 0].copy()
        return e
    _patch(monkeypatch, "cofem_estep", bad)
    _fails(TP.test_identity_dictionary_closed_form, "dense")
