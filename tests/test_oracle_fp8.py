"""The FP8 (OCP E4M3) dictionary for the mixed-precision E-step: the format
pinned code by code against its bit layout, and the measured contraction of
iterative refinement with an E4M3 inner operator at a scaled-down copy of the
dense 4096 x 16384 workload (same law: N = D/4, N(0, 1/N) entries, 1%
nonzeros, beta = 1e3).  The finding: with an E4M3 Phi the refinement
diverges in the first EM iterations (spectral radius of I - A~^-1 A above
one while alpha is small) and contracts only once the M-step has driven most
alpha up; bfloat16 contracts by ~0.15 from the start."""
import numpy as np
import pytest

import oracle as O
from oracle import lowprec as LP
from paper_2202_12808_amd import synth


def test_e4m3_every_code_round_trips():
    vals = [LP.decode_e4m3(c) for c in range(256)]
    finite = sorted({v for v in vals if v is not None})
    assert finite[-1] == 448.0 and finite[0] == -448.0
    assert min(v for v in finite if v > 0) == 2.0 ** -9
    for v in finite:
        assert LP.round_to_e4m3(np.array([v]))[0] == v
    # 254 finite codes, +0 and -0 the same value: 253 distinct values
    assert len(finite) == 253


def test_e4m3_rounding_ties_and_saturation():
    r = LP.round_to_e4m3
    pos = sorted(v for v in {LP.decode_e4m3(c) for c in range(128)} if v is not None)
    # midpoints between neighbours go to the one with an even mantissa code
    for a, b in zip(pos[:-1], pos[1:]):
        mid = 0.5 * (a + b)
        code_a = next(c for c in range(128) if LP.decode_e4m3(c) == a)
        want = a if code_a % 2 == 0 else b
        assert r(np.array([mid]))[0] == want, (a, b)
        assert r(np.array([np.nextafter(mid, a)]))[0] == a
        assert r(np.array([np.nextafter(mid, b)]))[0] == b
    assert r(np.array([1e6, -1e6, 470.0]))[0] == 448.0
    assert r(np.array([-1e6]))[0] == -448.0
    assert r(np.array([2.0 ** -11]))[0] == 0.0 and r(np.array([3 * 2.0 ** -11]))[0] == 2.0 ** -9


def test_contraction_pins():
    rng = np.random.default_rng(0)
    phi = rng.standard_normal((20, 40)) / np.sqrt(20)
    alpha = np.exp(rng.uniform(-1, 3, 40))
    assert LP.refinement_contraction(phi, phi, 50.0, alpha) < 1e-12
    # a uniformly scaled dictionary with alpha scaled alike: A~ = c A, radius |1 - 1/c|
    c = 1.7
    phi_c = phi * np.sqrt(c)
    A = 50.0 * phi.T @ phi + np.diag(alpha)
    At = 50.0 * phi_c.T @ phi_c + np.diag(alpha)
    ev = np.linalg.eigvals(np.linalg.solve(At, A)).real
    assert np.isclose(LP.refinement_contraction(phi, phi_c, 50.0, alpha), max(abs(1 - ev)), rtol=1e-9)


@pytest.fixture(scope="module")
def scaled_c2():
    p = synth.dense_problem(512, 2048, rho=0.01, beta=1e3, K=8, tol=1e-5, seed=0)
    phi = p.phi.astype(np.float64)
    phi8, scale = LP.e4m3_dictionary(phi)
    phi16 = synth.round_to_bf16(p.phi).astype(np.float64)
    op = O.DenseOperator(phi)
    alphas = {1: np.ones(p.D)}
    for T in (5, 12):
        alphas[T] = O.cofem(op, p.y, p.beta, T - 1, p.K, tol=p.tol, max_iter=400, seed=0).alpha
    return p, phi, phi8, phi16, alphas, scale


def test_e4m3_refinement_diverges_early_and_contracts_late(scaled_c2):
    p, phi, phi8, phi16, alphas, scale = scaled_c2
    assert scale == 2.0 ** np.floor(np.log2(448.0 / np.abs(phi).max()))
    rel8 = np.linalg.norm(phi8 - phi) / np.linalg.norm(phi)
    rel16 = np.linalg.norm(phi16 - phi) / np.linalg.norm(phi)
    assert 0.01 < rel8 < 0.05 and rel16 < 3e-3
    rho = {(t, n): LP.refinement_contraction(phi, f, p.beta, a)
           for t, a in alphas.items() for n, f in (("fp8", phi8), ("bf16", phi16))}
    print({f"t={t} {n}": round(v, 3) for (t, n), v in rho.items()})
    assert rho[(1, "fp8")] > 1.5          # diverges at alpha = 1
    assert rho[(1, "bf16")] < 0.25        # bfloat16 contracts from the start
    assert rho[(1, "fp8")] > rho[(5, "fp8")] > rho[(12, "fp8")]
    assert rho[(12, "fp8")] < 1.0         # contracts once most alpha are large
    assert all(rho[(t, "bf16")] < 0.25 for t in alphas)


# ------------------------------------------------------------------ bf16 taps
def _dense_conv(taps, H, W):
    op = O.ConvOperator(np.asarray(taps, np.float64), H, W)
    return op.apply(np.eye(H * W))


def test_conv_contraction_pins():
    from oracle.lowprec import conv_refinement_contraction, refinement_contraction
    rng = np.random.default_rng(12)
    # the Fourier-domain formula against the dense eigen-decomposition
    for H, W, k in ((8, 8, 3), (6, 10, 5)):
        taps = rng.standard_normal((k, k))
        low = taps + 1e-2 * rng.standard_normal((k, k))
        for a in (0.5, 7.0):
            r = conv_refinement_contraction(taps, low, H, W, 30.0, a)
            ref = refinement_contraction(_dense_conv(taps, H, W), _dense_conv(low, H, W), 30.0, np.full(H * W, a))
            assert abs(r - ref) <= 1e-10 * max(ref, 1.0)
    # closed form of a 1 x 1 kernel: |beta (c~^2 - c^2)| / (beta c~^2 + a)
    r = conv_refinement_contraction(np.array([[1.5]]), np.array([[1.25]]), 4, 4, 2.0, 3.0)
    assert np.isclose(r, 2.0 * abs(1.25 ** 2 - 1.5 ** 2) / (2.0 * 1.25 ** 2 + 3.0))


def test_bf16_taps_refinement_contracts_on_the_9x9_law():
    # A refinement whose inner solves used the 9x9 taps rounded to bfloat16
    # would converge on the 9x9 kernel law of the 1024 x 1024 workload (beta =
    # 1e4, here on a 256 x 256 grid): the contraction at
    # alpha = 1 (the first E-step) is 0.17..0.35 and falls as alpha grows.
    from oracle.lowprec import conv_refinement_contraction
    from paper_2202_12808_amd import synth
    for seed in (0, 1, 2):
        p = synth.conv_problem(256, 256, 9, rho=0.01, beta=1e4, K=4, tol=1e-5, seed=seed)
        low = synth.round_to_bf16(p.taps)
        r = [conv_refinement_contraction(p.taps, low, 256, 256, p.beta, a) for a in (1.0, 10.0, 100.0)]
        print("bf16-taps contraction, seed", seed, "alpha 1/10/100:", r)
        assert 0.1 < r[0] < 0.5 and r[2] < r[1] < r[0]
