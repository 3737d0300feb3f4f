"""GPU tests of the persistent warp-specialised fused CG iteration of the
convolution dictionary (kernels_conv_ws.hip), through the C ABI.

The library picks it for large problems; COFEM_CONV_KERNEL=ws forces it (and
=tile the per-tile kernel) at context creation, so small, ragged and
several-task shapes run it here:

* against the per-tile kernel, launch for launch: a solve stopped after the
  operator pass and one fused iteration leaves bit-equal float probe columns
  (both kernels do the same per-element arithmetic) and float64 mean columns
  and residual norms equal to rounding (the fused launch's partial sums are
  added in another order).  Over a whole solve that order moves the float64
  step scalars by an ulp, which now and then moves a float32 scalar by one
  and the two float32 CG runs part (a few iterations apart at the stop), so
  whole solves are checked against the oracle instead;
* against the float64 oracle: one teacher-forced step at the GPU's CG count
  (plain CG, warm-started Jacobi PCG, and three tasks sharing alpha), at the
  1e-4 norm-wise and 1e-3 element-wise bars of the other step tests;
* bit-reproducible runs (every sum is reduced in a fixed order);
* the operator alone (the apply mode): bit-equal to the per-tile kernel's q
  and within the float32 rounding bound of the float64 oracle's A v, element
  by element;
* a warm-started E-step (its start in the init mode, R = B - A X0 and
  P = M^-1 R formed in the launch, and its true residual in the residual
  mode): launch for launch as the per-tile kernels, two float64 tasks
  included;
* grids other than one workgroup per compute unit (the single-level finish
  ticket, several units per step).

The full-size 1024 x 1024 step tests (test_gpu_fullsize.py) run it too, since
the library chooses it there.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from oracle import multitask as M
from paper_2202_12808_amd import synth

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-4
ELEM_TOL = 1e-3


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def maxerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    m = float(np.abs(b).max())
    return float(np.abs(a - b).max() / (m if m > 0 else 1.0))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12808_amd import cofem as C
    C.load()
    return torch


class _kernel:
    """COFEM_CONV_KERNEL for the contexts created inside the block."""

    def __init__(self, mode):
        self.mode = mode

    def __enter__(self):
        self.old = os.environ.get("COFEM_CONV_KERNEL")
        os.environ["COFEM_CONV_KERNEL"] = self.mode

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("COFEM_CONV_KERNEL", None)
        else:
            os.environ["COFEM_CONV_KERNEL"] = self.old


def _ctx(torch, p, **kw):
    from paper_2202_12808_amd.cofem import CoFEM
    y = torch.from_numpy(np.ascontiguousarray(p.y)).cuda()
    return CoFEM.conv(torch.from_numpy(p.taps).cuda(), y, p.H, p.W, p.beta, p.K, tol=p.tol, max_iter=p.max_iter,
                      seed=p.seed, **kw)


_SHAPES = {
    # (problem, context options)
    "256x256_k9_K16": (lambda: synth.conv_problem(256, 256, 9, rho=0.01, beta=100.0, K=16, tol=1e-5, seed=11), {}),
    "200x328_k5_K5_ragged": (lambda: synth.conv_problem(200, 328, 5, rho=0.02, beta=1e3, K=5, tol=1e-5, seed=12),
                             {"jacobi": True, "warm_start": True}),
    "136x72_k9_K3": (lambda: synth.conv_problem(136, 72, 9, rho=0.03, beta=1e3, K=3, tol=1e-5, seed=13),
                     {"jacobi": True}),
    "96x160_k5_T3": (lambda: synth.conv_multitask(96, 160, 5, 3, rho=0.02, beta=1e3, K=6, tol=1e-5, seed=14),
                     {"jacobi": True, "warm_start": True}),
}


def _one_fused(torch, p, kw, mode):
    """The first E-step stopped after two CG iterations (the operator pass,
    then one fused launch): probe block, mean columns, residual ratio."""
    with _kernel(mode):
        with _ctx(torch, p, **kw) as g:
            g.set_fixed_cg_iters(2)
            st = g.em_step(1)[0]
            X, _ = g.solution()
            means = g.means().cpu().numpy().astype(np.float64)
    return X.cpu().numpy(), means, st["rel_resid"]


@pytest.mark.parametrize("case", sorted(_SHAPES))
def test_ws_launch_matches_tile_kernel(torch_dev, case):
    torch = torch_dev
    mk, kw = _SHAPES[case]
    p = mk()
    _say("ws vs tile launch", case)
    X_t, m_t, r_t = _one_fused(torch, p, kw, "tile")
    X_w, m_w, r_w = _one_fused(torch, p, kw, "ws")
    _say(case, "probe entries differing", int((X_t != X_w).sum()), "mean relerr", relerr(m_w, m_t),
         "ratio", r_t, r_w)
    assert np.array_equal(X_w, X_t)
    assert relerr(m_w, m_t) < 1e-13
    assert abs(r_w - r_t) <= 1e-12 * r_t


def _two_steps(torch, p, kw, mode, alpha):
    """The first E-step (alpha = 1), then one from `alpha`."""
    with _kernel(mode):
        with _ctx(torch, p, **kw) as g:
            first = g.em_step(1)[0]["cg_iters"]
            g.set_alpha(torch.from_numpy(alpha).cuda())
            st = g.em_step(1)[0]
            X, _ = g.solution()
            means = g.means().cpu().numpy().astype(np.float64)
    return (first, st["cg_iters"]), X.cpu().numpy(), means


def test_ws_runs_are_bit_reproducible(torch_dev):
    torch = torch_dev
    p = synth.conv_problem(200, 328, 5, rho=0.02, beta=1e3, K=5, tol=1e-5, seed=12)
    kw = {"jacobi": True, "warm_start": True}
    alpha = np.exp(np.random.default_rng(6).uniform(np.log(1e-2), np.log(1e3), p.D)).astype(np.float32)
    runs = [_two_steps(torch, p, kw, "ws", alpha) for _ in range(2)]
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])


@pytest.mark.parametrize("mode", ["plain", "warm_jacobi"])
def test_ws_step_parity(torch_dev, mode):
    # a ragged image (partial tiles on both edges) with the persistent kernel
    # forced; the oracle replays the step at the GPU's CG count
    torch = torch_dev
    beta = 1e3 if mode == "warm_jacobi" else 100.0
    p = synth.conv_problem(200, 328, 5, rho=0.02, beta=beta, K=5, tol=1e-5, seed=12)
    op = O.ConvOperator(p.taps.astype(np.float64), p.H, p.W)
    b0 = p.beta * op.apply_t(p.y.astype(np.float64))
    kw = {"jacobi": True, "warm_start": True} if mode == "warm_jacobi" else {}
    _say("ws step parity", mode)
    with _kernel("ws"):
        with _ctx(torch, p, **kw) as g:
            g.em_step(3)
            _, s_prev, alpha = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
            mu_prev = g.solution()[1].cpu().numpy()
            if not kw:  # plain CG: the step at a fixed 30 iterations (as the full-size test)
                g.set_fixed_cg_iters(30)
            st = g.em_step(1)[0]
            mu, s, a = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
    if kw:
        hh = float(np.sum(p.taps.astype(np.float64) ** 2))
        minv = (1.0 / (p.beta * hh + alpha)).astype(np.float32).astype(np.float64)
        e = O.cofem_estep_pcg(op, b0, p.beta, alpha, p.K, p.tol, p.max_iter, p.seed, st["t"], minv=minv,
                              mu0=mu_prev, d0=np.maximum(s_prev, 0.0), fixed_iters=st["cg_iters"])
    else:
        e = O.cofem_estep(op, b0, p.beta, alpha, p.K, p.tol, p.max_iter, p.seed, st["t"],
                          fixed_iters=st["cg_iters"])
    a_ref, _ = O.mstep(e.mu, e.s)
    got, ref = (mu, s, 1.0 / a), (e.mu, e.s, 1.0 / a_ref)
    errs = [relerr(x, y) for x, y in zip(got, ref)]
    elem = [maxerr(x, y) for x, y in zip(got, ref)]
    _say("ws", mode, "t", st["t"], "cg", st["cg_iters"], "relerr", errs, "max-entry", elem)
    assert st["cg_iters"] >= 2  # fused iterations ran
    assert all(x < STEP_TOL for x in errs), errs
    assert all(x < ELEM_TOL for x in elem), elem


def test_ws_multitask_step_parity(torch_dev):
    # three tasks sharing alpha: twelve float64 quadrant units per tile ahead
    # of the float tiles; the oracle's PCG replays the warm-started step
    torch = torch_dev
    p = synth.conv_multitask(96, 160, 5, 3, rho=0.02, beta=1e3, K=6, tol=1e-5, seed=14)
    op = O.ConvOperator(p.taps.astype(np.float64), p.H, p.W)
    B0 = p.beta * op.apply_t(p.y.T.astype(np.float64))
    _say("ws multitask step parity")
    with _kernel("ws"):
        with _ctx(torch, p, jacobi=True, warm_start=True) as g:
            g.em_step(3)
            _, s_prev, alpha = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
            mu_prev = g.means().cpu().numpy().T
            st = g.em_step(1)[0]
            _, s, a_new = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
            mu = g.means().cpu().numpy().T
    hh = float(np.sum(p.taps.astype(np.float64) ** 2))
    minv = (1.0 / (p.beta * hh + alpha)).astype(np.float32).astype(np.float64)
    P = O.rademacher_probes(p.seed, st["t"], p.K, p.D)
    X0 = np.concatenate([np.maximum(s_prev, 0.0)[:, None] * P, mu_prev], axis=1)
    X, _ = O.pcg_solve(O.make_apply_A(op, p.beta, alpha), np.concatenate([P, B0], axis=1), p.tol, p.max_iter, minv,
                       X0, st["cg_iters"])
    mu_ref, s_ref = X[:, p.K:], O.diag_estimate(P, X[:, :p.K])
    a_ref, _ = M.mstep_mt(mu_ref, s_ref)
    errs = (relerr(mu, mu_ref), relerr(s, s_ref), relerr(1.0 / a_new, 1.0 / a_ref))
    _say("ws multitask cg", st["cg_iters"], "relerr mu/s/(1/alpha)", errs)
    assert st["converged"] == 1
    assert all(e < STEP_TOL for e in errs), errs
    assert max(relerr(mu[:, j], mu_ref[:, j]) for j in range(3)) < STEP_TOL


_APPLY_SHAPES = {
    "256x256_k9_K16": (256, 256, 9, 16),
    "200x328_k5_K5_ragged": (200, 328, 5, 5),
    "136x72_k9_K3": (136, 72, 9, 3),
    "64x64_k1_K4": (64, 64, 1, 4),
}


@pytest.mark.parametrize("case", sorted(_APPLY_SHAPES))
def test_ws_apply_matches_tile_and_oracle(torch_dev, case):
    torch = torch_dev
    H, W, k, K = _APPLY_SHAPES[case]
    p = synth.conv_problem(H, W, k, rho=0.05, beta=321.0, K=K, tol=1e-6, seed=H * W + k)
    rng = np.random.default_rng(21)
    D = H * W
    alpha = (10.0 ** rng.uniform(-2, 6, D)).astype(np.float32)
    V = rng.standard_normal((D, K)).astype(np.float32)
    vm = rng.standard_normal(D)
    _say("ws apply", case)
    out = {}
    for mode in ("tile", "ws"):
        with _kernel(mode):
            with _ctx(torch, p) as g:
                g.set_alpha(torch.from_numpy(alpha))
                q, qm = g.apply_A(torch.from_numpy(V.T.copy()), torch.from_numpy(vm))
                out[mode] = (q.cpu().numpy().T, qm.cpu().numpy())
    assert np.array_equal(out["ws"][0], out["tile"][0])
    assert relerr(out["ws"][1], out["tile"][1]) < 1e-15
    op = O.ConvOperator(p.taps.astype(np.float64), H, W)
    A = O.make_apply_A(op, p.beta, alpha.astype(np.float64))
    ref = A(V.astype(np.float64))
    # element-wise: float32 rounding of the two stencil stages, relative to
    # the magnitudes that enter each output (beta |Phi|^T |Phi| |v| + alpha |v|)
    habs = O.ConvOperator(np.abs(p.taps.astype(np.float64)), H, W)
    scale = p.beta * habs.apply_t(habs.apply(np.abs(V.astype(np.float64)))) + alpha[:, None] * np.abs(V)
    err = np.abs(out["ws"][0] - ref) / scale
    _say(case, "max error / magnitude", float(err.max()))
    assert float(err.max()) < (2 * k * k + 4) * 2 ** -23
    assert relerr(out["ws"][1], A(vm)) < 1e-13


@pytest.mark.parametrize("grid", [100, 64])
def test_ws_other_grids_match_tile_kernel(torch_dev, grid):
    # a grid that is not a multiple of 8 takes the single-level finish ticket
    # and the plain slot order; 64 workgroups take several units per step
    torch = torch_dev
    mk, kw = _SHAPES["200x328_k5_K5_ragged"]
    p = mk()
    _say("ws grid", grid)
    X_t, m_t, r_t = _one_fused(torch, p, kw, "tile")
    X_w, m_w, r_w = _one_fused(torch, p, kw, f"ws:{grid}")
    assert np.array_equal(X_w, X_t)
    assert relerr(m_w, m_t) < 1e-13
    assert abs(r_w - r_t) <= 1e-12 * r_t


def _warm_second_step(torch, p, kw, mode):
    """A first E-step, then a warm-started second one, both stopped after two
    CG iterations: the second starts with the init mode (R, P from A X0) and
    ends with the residual mode (the true residual)."""
    with _kernel(mode):
        with _ctx(torch, p, **kw) as g:
            g.set_fixed_cg_iters(2)
            g.em_step(1)
            st = g.em_step(1)[0]
            X, _ = g.solution()
            means = g.means().cpu().numpy().astype(np.float64)
    return X.cpu().numpy(), means, st["rel_resid"]


@pytest.mark.parametrize("case", ["200x328_k5_K5_ragged", "96x160_k5_T3"])
def test_ws_warm_start_and_residual_match_tile_kernel(torch_dev, case):
    torch = torch_dev
    mk, kw = _SHAPES[case]
    p = mk()
    assert kw.get("warm_start")
    _say("ws warm start + residual vs tile", case)
    X_t, m_t, r_t = _warm_second_step(torch, p, kw, "tile")
    X_w, m_w, r_w = _warm_second_step(torch, p, kw, "ws")
    _say(case, "probe entries differing", int((X_t != X_w).sum()), "mean relerr", relerr(m_w, m_t), "ratio", r_t, r_w)
    assert np.array_equal(X_w, X_t)
    assert relerr(m_w, m_t) < 1e-13
    assert abs(r_w - r_t) <= 1e-12 * r_t


def test_ws_residual_launched_ahead_of_the_stop_read(torch_dev):
    # With the true residual on, the persistent kernel's residual is the launch
    # enqueued ahead of a predicted solve's first poll, and it runs only if the
    # solve has stopped by then.  Both outcomes: warm-started EM iterations whose
    # counts fall (that launch is the residual), then set_alpha to another wide
    # alpha, whose solve from the previous solution needs more iterations than
    # the last one (that launch does nothing; the residual follows the stop).
    # Against the per-tile path, which computes the residual in its own
    # launches after the stop.
    torch = torch_dev
    p = synth.conv_problem(200, 328, 5, rho=0.02, beta=1e3, K=5, tol=1e-5, seed=12)
    kw = {"jacobi": True, "warm_start": True}
    a1, a2 = (np.exp(np.random.default_rng(s).uniform(np.log(1e-2), np.log(1e3), p.D)).astype(np.float32)
              for s in (6, 7))
    runs = {}
    for mode in ("tile", "ws"):
        with _kernel(mode):
            with _ctx(torch, p, **kw) as g:
                st = g.em_step(1)
                g.set_alpha(torch.from_numpy(a1).cuda())
                st += g.em_step(3)
                g.set_alpha(torch.from_numpy(a2).cuda())
                st += g.em_step(1)
                runs[mode] = st
                X, _ = g.solution()
                runs[mode + "_X"] = X.cpu().numpy()
    cg = [x["cg_iters"] for x in runs["ws"]]
    _say("cg ws", cg, "tile", [x["cg_iters"] for x in runs["tile"]],
         "true ratios ws", [x["rel_resid_true"] for x in runs["ws"]],
         "tile", [x["rel_resid_true"] for x in runs["tile"]])
    assert all(cg[i] <= cg[i - 1] for i in range(1, 4))  # the launch ahead found the solve stopped
    assert cg[4] > cg[3]  # ... and running
    assert cg == [x["cg_iters"] for x in runs["tile"]]
    # (the two paths' float64 sums differ in order, so over several EM
    # iterations a float32 alpha may round differently at some pixel: ratios to
    # 1e-6; a residual taken before the last update, or one left from the
    # previous E-step, is off by far more)
    for w, t in zip(runs["ws"], runs["tile"]):
        assert w["rel_resid_true"] > 0.0
        assert abs(w["rel_resid_true"] - t["rel_resid_true"]) <= 1e-6 * t["rel_resid_true"]
        assert abs(w["rel_resid"] - t["rel_resid"]) <= 1e-6 * t["rel_resid"]
    assert relerr(runs["ws_X"], runs["tile_X"]) < 1e-5
