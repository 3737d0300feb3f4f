"""GPU tests of the spectral start (COFEM_FLAG_SPECTRAL_START) through the C
ABI: the first E-step of a circular-convolution problem (alpha = 1, so A is
block-circulant) starts from the 2D-DFT solve of A X = B and CG's stop test
judges it.  References are the oracle's exact Fourier-domain solve
(ConvOperatorFFT.solve_shifted, pinned against the direct stencil and dense
Cholesky solves) and its spectral-start EM (cofem(spectral_start=True))."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2202_12808_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12808_amd import cofem as C
    C.load()
    return torch


def _conv(torch, p, y=None, **kw):
    from paper_2202_12808_amd.cofem import CoFEM
    y = torch.from_numpy(p.y if y is None else y).cuda()
    return CoFEM.conv(torch.from_numpy(p.taps).cuda(), y, p.H, p.W, p.beta, p.K, tol=p.tol,
                      max_iter=p.max_iter, seed=p.seed, **kw)


def _exact_first_estep(p, t=1, Y=None):
    """[P | b0_1 .. b0_T] and its exact solve at alpha = 1 (float64 DFTs)."""
    fft = O.ConvOperatorFFT(p.taps.astype(np.float64), p.H, p.W)
    Y = np.asarray(p.y if Y is None else Y, np.float64).reshape(-1, p.D)
    B0 = p.beta * fft.apply_t(Y.T)
    P = O.rademacher_probes(p.seed, t, p.K, p.D)
    B = np.concatenate([P, B0], axis=1)
    return fft, B, fft.solve_shifted(B, p.beta, 1.0)


def _true_resid(fft, beta, X, B):
    R = B - (beta * fft.gram(X) + X)
    return float(np.linalg.norm(R) / np.linalg.norm(B))


# the start's float32 rounding leaves a residual near 1e-6 to 1e-5 relative
# (the transforms' rounding times the spread of lambda); the solve then takes
# at most a few CG iterations, where zero-started CG needs hundreds
_CASES = {
    "64x128_k7": (lambda: synth.conv_problem(64, 128, 7, rho=0.02, beta=1e3, K=8, tol=1e-6, seed=3), 4),
    "128x32_k9_K5": (lambda: synth.conv_problem(128, 32, 9, rho=0.02, beta=1e4, K=5, tol=1e-5, seed=4), 4),
    "256x256_k7": (lambda: synth.conv_problem(256, 256, 7, rho=0.02, beta=1e4, K=16, tol=1e-5, seed=5,
                                              law="laplace"), 4),
    "1x256_k3": (lambda: synth.conv_problem(1, 256, 3, rho=0.05, beta=1e3, K=4, tol=1e-6, seed=6), 4),
}


@pytest.mark.parametrize("case", sorted(_CASES))
def test_first_estep_matches_exact_solve(torch_dev, case):
    torch = torch_dev
    mk, max_cg = _CASES[case]
    p = mk()
    fft, B, Xe = _exact_first_estep(p)
    _say("spectral first E-step", case)
    with _conv(torch, p, spectral_start=True, jacobi=True, warm_start=True) as g:
        st = g.em_step(1)[0]
        probes, mean = g.solution()
        mu, s, _ = g.posterior()
    X = np.concatenate([probes.cpu().numpy().astype(np.float64).T, mean.cpu().numpy()[:, None]], axis=1)
    mu = mu.cpu().numpy().astype(np.float64)
    s = s.cpu().numpy().astype(np.float64)
    s_exact = O.diag_estimate(B[:, :p.K], Xe[:, :p.K])
    tr = _true_resid(fft, p.beta, X, B)
    errs = (relerr(X[:, p.K], Xe[:, p.K]), relerr(s, s_exact), relerr(X[:, :p.K], Xe[:, :p.K]))
    _say(case, "cg", st["cg_iters"], "gpu true resid", st["rel_resid_true"], "fp64 true resid", tr,
         "relerr mu/s/X", errs)
    assert st["converged"] and st["cg_iters"] <= max_cg
    # the solve's own test holds on the recursive residual; the true residual
    # of the returned block, in float64, is at the float32 floor
    assert tr < 3 * p.tol + 2e-5
    assert errs[0] < 1e-4 and errs[1] < 1e-4 and errs[2] < 1e-4
    # element-wise: every mean entry within 1e-4 of the largest
    assert np.max(np.abs(X[:, p.K] - Xe[:, p.K])) <= 1e-4 * np.max(np.abs(Xe[:, p.K]))
    assert np.allclose(mu, X[:, p.K], rtol=1e-6, atol=1e-7 * np.max(np.abs(mu)))


def test_first_estep_fp64_mode(torch_dev):
    # float64 probe columns: the float32 start (residual near 1e-7) leaves the
    # solve a smaller reduction to make than a zero start; it then reaches the
    # float64 tolerance as usual
    torch = torch_dev
    p = synth.conv_problem(32, 64, 5, rho=0.03, beta=1e3, K=6, tol=1e-10, seed=8)
    fft, B, Xe = _exact_first_estep(p)
    _say("spectral first E-step, float64 probes")
    with _conv(torch, p, jacobi=True, precision="fp64") as g:
        cold = g.em_step(1)[0]
    with _conv(torch, p, spectral_start=True, jacobi=True, precision="fp64") as g:
        st = g.em_step(1)[0]
        mean = g.solution()[1].cpu().numpy()
    r_mean = np.linalg.norm(B[:, p.K] - (p.beta * fft.gram(mean) + mean)) / np.linalg.norm(B)
    _say("fp64: cg", st["cg_iters"], "zero start", cold["cg_iters"], "device true resid", st["rel_resid_true"],
         "mean column resid", r_mean, "relerr mean", relerr(mean, Xe[:, p.K]))
    assert st["converged"] and st["cg_iters"] < cold["cg_iters"]
    # the device's float64 true residual over all columns, and the float64
    # mean column's share of it, evaluated by the oracle
    assert st["rel_resid_true"] < 3 * p.tol
    assert r_mean < 3 * p.tol
    assert relerr(mean, Xe[:, p.K]) < 1e-7


def test_multitask_first_estep(torch_dev):
    torch = torch_dev
    p = synth.conv_multitask(64, 64, 5, 3, rho=0.02, beta=1e3, K=7, tol=1e-6, seed=9)
    fft, B, Xe = _exact_first_estep(p, Y=p.y)
    _say("spectral first E-step, T = 3, K = 7 (odd column count)")
    with _conv(torch, p, spectral_start=True, jacobi=True) as g:
        st = g.em_step(1)[0]
        means = g.means().cpu().numpy()
        probes = g.solution()[0].cpu().numpy().astype(np.float64).T
    errs = [relerr(means[t], Xe[:, p.K + t]) for t in range(3)]
    _say("multitask: cg", st["cg_iters"], "relerr means", errs, "probes", relerr(probes, Xe[:, :p.K]))
    assert st["converged"] and st["cg_iters"] <= 4
    assert max(errs) < 1e-4 and relerr(probes, Xe[:, :p.K]) < 1e-4


def test_trajectory_matches_oracle(torch_dev):
    # three EM iterations of the spectral-start control form against the
    # oracle's (float64 start, then warm-started Jacobi PCG)
    torch = torch_dev
    p = synth.conv_problem(64, 64, 7, rho=0.02, beta=1e3, K=8, tol=1e-7, seed=12)
    op = O.ConvOperatorFFT(p.taps.astype(np.float64), p.H, p.W)
    ref = O.cofem(op, p.y.astype(np.float64), p.beta, 3, p.K, tol=p.tol, max_iter=p.max_iter, seed=p.seed,
                  warm_start=True, jacobi=True, spectral_start=True)
    with _conv(torch, p, spectral_start=True, jacobi=True, warm_start=True) as g:
        stats = g.em_step(3)
        mu, s, alpha = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
    its = [st["cg_iters"] for st in stats]
    errs = (relerr(mu, ref.mu), relerr(s, ref.s), relerr(1.0 / alpha, 1.0 / ref.alpha))
    _say("trajectory: cg gpu", its, "oracle", [st["cg_iters"] for st in ref.stats], "relerr", errs)
    assert ref.stats[0]["cg_iters"] == 0 and its[0] <= 4
    for a, b in zip(its[1:], ref.stats[1:]):
        assert abs(a - b["cg_iters"]) <= max(2, 0.2 * b["cg_iters"])
    assert all(e < 1e-3 for e in errs)


def test_restart_and_set_alpha(torch_dev):
    # cofem_restart brings back alpha = 1 and the spectral start (bit for bit
    # a fresh context); after cofem_set_alpha the first solve starts cold
    torch = torch_dev
    p = synth.conv_problem(64, 32, 5, rho=0.03, beta=1e3, K=6, tol=1e-6, seed=13)
    kw = dict(spectral_start=True, jacobi=True, warm_start=True)
    with _conv(torch, p, **kw) as g:
        a = g.em_step(3)
        mu_a = g.posterior()[0].cpu().numpy()
        g.restart()
        b = g.em_step(3)
        mu_b = g.posterior()[0].cpu().numpy()
        ones = torch.ones(p.D, dtype=torch.float32, device="cuda")
        g.restart()
        g.set_alpha(ones)
        c = g.em_step(1)[0]
    _say("restart: cg", [x["cg_iters"] for x in a], [x["cg_iters"] for x in b], "after set_alpha", c["cg_iters"])
    assert [x["cg_iters"] for x in a] == [x["cg_iters"] for x in b]
    assert np.array_equal(mu_a, mu_b)
    assert a[0]["cg_iters"] <= 4 and c["cg_iters"] > 3 * a[0]["cg_iters"] + 10


def test_rejections(torch_dev):
    torch = torch_dev
    from paper_2202_12808_amd.cofem import CofemError, CoFEM
    p = synth.conv_problem(48, 64, 5, rho=0.03, beta=1e3, K=4, tol=1e-6, seed=14)
    with pytest.raises(CofemError, match="power-of-two"):
        _conv(torch, p, spectral_start=True)
    d = synth.dense_problem(64, 128, nnz=4, beta=1e3, K=4, tol=1e-6, seed=14)
    with pytest.raises(CofemError, match="convolution"):
        CoFEM.dense(torch.from_numpy(d.phi).cuda(), torch.from_numpy(d.y).cuda(), d.beta, d.K,
                    spectral_start=True)


def test_fullsize_1024_k9(torch_dev):
    # the 1024 x 1024, 9 x 9, K = 16, beta = 1e4 workload: the first E-step
    # against the exact solve (17 float64 2D DFT pairs on the host)
    torch = torch_dev
    p = synth.WORKLOADS["conv_1024x1024_k9"](0)
    fft, B, Xe = _exact_first_estep(p)
    _say("spectral first E-step at 1024x1024, K =", p.K)
    with _conv(torch, p, spectral_start=True, jacobi=True, warm_start=True) as g:
        st = g.em_step(1)[0]
        probes, mean = g.solution()
    X = np.concatenate([probes.cpu().numpy().astype(np.float64).T, mean.cpu().numpy()[:, None]], axis=1)
    tr = _true_resid(fft, p.beta, X, B)
    errs = (relerr(X[:, p.K], Xe[:, p.K]), relerr(X[:, :p.K], Xe[:, :p.K]))
    worst = np.max(np.abs(X[:, p.K] - Xe[:, p.K])) / np.max(np.abs(Xe[:, p.K]))
    _say("1024: cg", st["cg_iters"], "true resid", tr, "relerr mean/probes", errs, "max elem", worst)
    assert st["converged"] and st["cg_iters"] <= 6
    assert tr < 3 * p.tol + 2e-5
    assert errs[0] < 1e-3 and errs[1] < 1e-3 and worst < 1e-3
