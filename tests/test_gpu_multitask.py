"""Multi-task SBL (the extension Sec. 5 names: T observation vectors sharing
alpha) on the convolution and dense dictionaries, through the C ABI, against the float64
multi-task oracle: one teacher-forced E-step + M-step at the GPU's CG count,
with and without the warm-started Jacobi form, and the true residual of
every task's column."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import multitask as M
from paper_2202_12808_amd import synth

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-4


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12808_amd import cofem as C
    C.load()
    return torch


def _ctx(torch, p, **kw):
    from paper_2202_12808_amd.cofem import CoFEM
    Y = torch.from_numpy(np.ascontiguousarray(p.y)).cuda()
    if p.kind == "conv":
        return CoFEM.conv(torch.from_numpy(p.taps).cuda(), Y, p.H, p.W, p.beta, p.K, tol=p.tol,
                          max_iter=p.max_iter, seed=p.seed, **kw)
    return CoFEM.dense(torch.from_numpy(p.phi).cuda(), Y, p.beta, p.K, tol=p.tol, max_iter=p.max_iter,
                       seed=p.seed, **kw)


def _op(p):
    if p.kind == "conv":
        return O.ConvOperator(p.taps.astype(np.float64), p.H, p.W)
    return O.DenseOperator(p.phi.astype(np.float64))


_CASES = {
    "dense_T2": (lambda: synth.dense_multitask(256, 1024, 2, rho=0.02, beta=1e4, K=20, tol=1e-6, seed=5), {}),
    "dense_T4_ragged": (lambda: synth.dense_multitask(300, 777, 4, rho=0.02, beta=5e3, K=13, tol=1e-6, seed=6), {}),
    "dense_T3_split": (lambda: synth.dense_multitask(512, 8192, 3, rho=0.02, beta=1e3, K=32, tol=1e-5, seed=7), {}),
    "conv_T3": (lambda: synth.conv_multitask(64, 48, 7, 3, rho=0.02, beta=100.0, K=8, tol=1e-6, seed=5), {}),
    "conv_T4_jacobi_warm": (lambda: synth.conv_multitask(40, 52, 5, 4, rho=0.03, beta=1e3, K=6, tol=1e-5, seed=6),
                            {"jacobi": True, "warm_start": True}),
    "conv_T2_fp64": (lambda: synth.conv_multitask(48, 40, 7, 2, rho=0.02, beta=1e4, K=8, tol=1e-6, seed=7),
                     {"precision": "fp64"}),
}


@pytest.mark.parametrize("case", sorted(_CASES))
def test_multitask_step_parity(torch_dev, case):
    torch = torch_dev
    mk, kw = _CASES[case]
    p = mk()
    T = p.tasks
    op = _op(p)
    B0 = p.beta * op.apply_t(p.y.T.astype(np.float64))
    pcg = kw.get("jacobi") or kw.get("warm_start")
    _say("multitask case", case, "kind", p.kind, "T", T, "D", p.D, "K", p.K)
    with _ctx(torch, p, **kw) as g:
        g.em_step(3)
        _, s_prev, alpha = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
        mu_prev = g.means().cpu().numpy().T
        st = g.em_step(1)[0]
        _, s, a_new = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
        mu = g.means().cpu().numpy().T
    t = st["t"]
    if pcg:
        hh = float(np.sum(p.taps.astype(np.float64) ** 2))
        minv = (1.0 / (p.beta * hh + alpha)).astype(np.float32).astype(np.float64)
        P = O.rademacher_probes(p.seed, t, p.K, p.D)
        X0 = np.concatenate([np.maximum(s_prev, 0.0)[:, None] * P, mu_prev], axis=1)
        X, _ = O.pcg_solve(O.make_apply_A(op, p.beta, alpha), np.concatenate([P, B0], axis=1), p.tol, p.max_iter,
                           minv, X0, st["cg_iters"])
        mu_ref, s_ref = X[:, p.K:], O.diag_estimate(P, X[:, :p.K])
    else:
        e = M.cofem_estep_mt(op, B0, p.beta, alpha, p.K, p.tol, p.max_iter, p.seed, t, fixed_iters=st["cg_iters"])
        mu_ref, s_ref = e.mu, e.s
    a_ref, _ = M.mstep_mt(mu_ref, s_ref)
    errs = (relerr(mu, mu_ref), relerr(s, s_ref), relerr(1.0 / a_new, 1.0 / a_ref))
    per_task = [relerr(mu[:, j], mu_ref[:, j]) for j in range(T)]
    _say(case, "T", T, "t", t, "cg", st["cg_iters"], "relerr mu/s/(1/alpha)", errs, "per task", per_task)
    assert mu.shape == (p.D, T)
    assert st["converged"] == 1 or st["cg_iters"] == p.max_iter
    assert all(err < STEP_TOL for err in errs), errs
    assert max(per_task) < STEP_TOL


@pytest.mark.parametrize("kind", ["conv", "dense"])
def test_multitask_true_residual_covers_every_task(torch_dev, kind):
    torch = torch_dev
    p = (synth.conv_multitask(40, 36, 5, 3, rho=0.03, beta=1e3, K=8, tol=1e-5, seed=8) if kind == "conv"
         else synth.dense_multitask(200, 700, 3, rho=0.02, beta=1e3, K=10, tol=1e-5, seed=8))
    op = _op(p)
    B0 = p.beta * op.apply_t(p.y.T.astype(np.float64))
    with _ctx(torch, p) as g:
        g.em_step(2)
        alpha = g.posterior()[2].cpu().numpy().astype(np.float64)
        st = g.em_step(1)[0]
        X, _ = g.solution()
        mu = g.means().cpu().numpy().T
    X = np.concatenate([X.cpu().numpy().astype(np.float64).T, mu], axis=1)
    B = np.concatenate([O.rademacher_probes(p.seed, st["t"], p.K, p.D), B0], axis=1)
    ref = O.true_relative_residual(O.make_apply_A(op, p.beta, alpha), X, B)
    _say("multitask true residual gpu", st["rel_resid_true"], "float64 recomputation", ref)
    assert abs(st["rel_resid_true"] - ref) <= 0.05 * ref + 1e-7


@pytest.mark.parametrize("kind", ["conv", "dense"])
def test_one_task_array_equals_single_task(torch_dev, kind):
    # y given as a (1, N) array is the single-task problem, bit for bit
    torch = torch_dev
    p = (synth.conv_problem(40, 36, 5, rho=0.03, beta=1e3, K=6, tol=1e-5, seed=9) if kind == "conv"
         else synth.dense_problem(200, 700, nnz=8, beta=1e3, K=12, tol=1e-5, seed=9))
    outs = []
    for y in (p.y, p.y[None, :]):
        q = synth.Problem(**{**p.__dict__, "y": np.ascontiguousarray(y)})
        with _ctx(torch, q) as g:
            g.em_step(3)
            outs.append([x.cpu().numpy() for x in g.posterior()])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_dense_multitask_rejections(torch_dev):
    torch = torch_dev
    from paper_2202_12808_amd import cofem as C
    p = synth.dense_multitask(64, 128, 2, rho=0.05, beta=100.0, K=4, tol=1e-5, seed=1)
    for kw in ({"precision": "bf16_ir"}, {"warm_start": True}):
        with pytest.raises(C.CofemError) as ei:
            _ctx(torch, p, **kw)
        assert ei.value.status == C.COFEM_ERR_UNSUPPORTED
    p5 = synth.dense_multitask(64, 128, 5, rho=0.05, beta=100.0, K=4, tol=1e-5, seed=1)
    with pytest.raises(C.CofemError) as ei:
        _ctx(torch, p5)
    assert ei.value.status == C.COFEM_ERR_UNSUPPORTED
