"""GPU tests of the solver controls around the E-step (through the C ABI):
restarting a context, the per-column CG stop rule and the EM-level stop of
cofem_em_run, each against the float64 oracle or a fresh context."""
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


def _ctx(torch, p, **kw):
    from paper_2202_12808_amd.cofem import CoFEM
    y = torch.from_numpy(p.y).cuda()
    if p.kind == "dense":
        return CoFEM.dense(torch.from_numpy(p.phi).cuda(), y, p.beta, p.K, tol=p.tol, max_iter=p.max_iter,
                           seed=p.seed, **kw)
    if p.kind == "conv":
        return CoFEM.conv(torch.from_numpy(p.taps).cuda(), y, p.H, p.W, p.beta, p.K, tol=p.tol,
                          max_iter=p.max_iter, seed=p.seed, **kw)
    return CoFEM.dct(torch.from_numpy(p.rows).cuda(), y, p.D, p.beta, p.K, tol=p.tol, max_iter=p.max_iter,
                     seed=p.seed, **kw)


# ------------------------------------------------------------------ restart
_WARM_FORMS = {
    "dense_fp32_warm": (lambda: synth.dense_problem(200, 700, nnz=8, beta=1e3, K=12, tol=1e-5, seed=11),
                        {"warm_start": True}),
    "dense_bf16_ir_warm": (lambda: synth.dense_problem(200, 700, nnz=8, beta=1e3, K=12, tol=1e-5, seed=11),
                           {"precision": "bf16_ir", "warm_start": True}),
    "conv_warm_jacobi": (lambda: synth.conv_problem(40, 36, 5, rho=0.03, beta=1e3, K=8, tol=1e-5, seed=11),
                         {"warm_start": True, "jacobi": True}),
    "dct_warm_jacobi": (lambda: synth.dct_problem(4096, rho=0.04, beta=4e4, K=6, tol=1e-5, seed=11),
                        {"warm_start": True, "jacobi": True}),
}


@pytest.mark.parametrize("form", sorted(_WARM_FORMS))
def test_restart_equals_fresh_context(torch_dev, form):
    # a restarted context repeats a fresh context's run bit for bit: alpha = 1,
    # t = 1 and no warm start from the previous run's last E-step
    torch = torch_dev
    mk, kw = _WARM_FORMS[form]
    p = mk()
    _say("restart", form)
    with _ctx(torch, p, **kw) as g:
        st_fresh = g.em_step(4)
        post_fresh = [x.cpu().numpy() for x in g.posterior()]
        g.restart()
        st_again = g.em_step(4)
        post_again = [x.cpu().numpy() for x in g.posterior()]
        # set_iteration alone also drops the previous solution: the next solve is cold
        g.restart()
        g.em_step(1)
        g.set_iteration(1)
        g.set_alpha(torch.ones(p.D))
        st_cold = g.em_step(1)
    cg_f = [x["cg_iters"] for x in st_fresh]
    cg_a = [x["cg_iters"] for x in st_again]
    _say("cg fresh", cg_f, "restarted", cg_a, "cold after set_iteration", st_cold[0]["cg_iters"])
    assert cg_f == cg_a
    assert st_cold[0]["cg_iters"] == cg_f[0]
    for a, b in zip(post_fresh, post_again):
        assert np.array_equal(a, b)


# ------------------------------------------------------------------ per-column stop rule
def _per_column_parity(torch, p, label, **kw):
    op = (O.DenseOperator(p.phi.astype(np.float64)) if p.kind == "dense"
          else O.ConvOperator(p.taps.astype(np.float64), p.H, p.W) if p.kind == "conv"
          else O.DctMaskOperator(p.rows, p.D))
    b0 = p.beta * op.apply_t(p.y.astype(np.float64))
    with _ctx(torch, p, stop_rule="per_column", **kw) as g:
        g.em_step(2)
        alpha = g.posterior()[2].cpu().numpy().astype(np.float64)
        st = g.em_step(1)[0]
        mu, s, a_new = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
    e = O.cofem_estep(op, b0, p.beta, alpha, p.K, p.tol, p.max_iter, p.seed, st["t"], stop_rule="per_column")
    a_ref, _ = O.mstep(e.mu, e.s)
    errs = (relerr(mu, e.mu), relerr(s, e.s), relerr(1.0 / a_new, 1.0 / a_ref))
    _say(label, "cg gpu", st["cg_iters"], "oracle", e.cg.iters, "converged", st["converged"], e.cg.converged,
         "relerr mu/s/(1/alpha)", errs)
    # Both runs stop on their own per-column decisions (no teacher-forced
    # count: the columns freeze at different iterations).  Float32 probe
    # columns converge more slowly near tolerances of 1e-6 (Krylov
    # orthogonality decays faster in float32), so the GPU may need some more
    # iterations than the float64 oracle; both meet every column's tolerance.
    assert st["converged"] == int(e.cg.converged)
    assert e.cg.iters - 1 <= st["cg_iters"] <= 1.25 * e.cg.iters + 2
    assert all(err < 1e-4 for err in errs), errs
    # each column meets its own tolerance (the float64 mean column exactly;
    # float32 probe columns to their rounding)
    A = O.make_apply_A(op, p.beta, alpha)
    X = e.X
    B = np.concatenate([e.P, b0[:, None]], axis=1)
    own = np.linalg.norm(B - A(X), axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(own < 1.01 * p.tol) or st["cg_iters"] == p.max_iter
    return st, e


def test_per_column_stop_dense(torch_dev):
    p = synth.dense_problem(256, 1024, nnz=20, beta=1e4, K=20, tol=1e-6, seed=0)
    st, e = _per_column_parity(torch_dev, p, "dense 256x1024 per-column")
    # the joint rule stops earlier (the mean column dominates ||B||_F)
    with _ctx(torch_dev, p) as g:
        g.em_step(2)
        joint = g.em_step(1)[0]["cg_iters"]
    assert joint < st["cg_iters"]


def test_per_column_stop_ragged_dense(torch_dev):
    _per_column_parity(torch_dev, synth.dense_problem(300, 777, nnz=9, beta=5e3, K=13, tol=1e-6, seed=3),
                       "dense 300x777 per-column")


def test_per_column_stop_conv_pcg(torch_dev):
    # the conv form with the Jacobi preconditioner (zero start: the oracle's
    # per-column PCG then equals its per-column CG up to the diagonal)
    torch = torch_dev
    p = synth.conv_problem(64, 48, 7, rho=0.02, beta=100.0, K=8, tol=1e-6, seed=1, law="laplace")
    op = O.ConvOperator(p.taps.astype(np.float64), p.H, p.W)
    b0 = p.beta * op.apply_t(p.y.astype(np.float64))
    with _ctx(torch, p, stop_rule="per_column", jacobi=True) as g:
        g.em_step(2)
        alpha = g.posterior()[2].cpu().numpy().astype(np.float64)
        st = g.em_step(1)[0]
        mu, s, a_new = [x.cpu().numpy().astype(np.float64) for x in g.posterior()]
    minv = 1.0 / (p.beta * float(np.sum(p.taps.astype(np.float64) ** 2)) + alpha)
    e = O.cofem_estep_pcg(op, b0, p.beta, alpha, p.K, p.tol, p.max_iter, p.seed, st["t"], minv=minv,
                          stop_rule="per_column")
    errs = (relerr(mu, e.mu), relerr(s, e.s))
    _say("conv per-column jacobi: cg", st["cg_iters"], e.cg.iters, "relerr mu/s", errs)
    assert e.cg.iters - 1 <= st["cg_iters"] <= 1.25 * e.cg.iters + 2
    assert all(err < 1e-4 for err in errs)


def test_per_column_stop_dct(torch_dev):
    _per_column_parity(torch_dev, synth.dct_problem(4096, rho=0.04, beta=4e4, K=6, tol=1e-6, seed=2),
                       "dct 4096 per-column")


# ------------------------------------------------------------------ EM-level stop
def test_em_run_stops_like_closed_form(torch_dev):
    # Phi = I: the prior variances follow a scalar recursion per coordinate,
    # so the relative change of 1/alpha at every EM iteration is known in
    # closed form; cofem_em_run reports it and stops at the first iteration
    # below em_tol
    torch = torch_dev
    from paper_2202_12808_amd.cofem import CoFEM
    D, beta = 320, 40.0
    rng = np.random.default_rng(21)
    y = (rng.standard_normal(D) * np.where(rng.random(D) < 0.3, 3.0, 0.05)).astype(np.float32)
    yd = y.astype(np.float64)
    a, g_prev, changes = np.ones(D), np.ones(D), []
    for _ in range(60):
        mu = beta * yd / (beta + a)
        g = mu * mu + 1.0 / (beta + a)
        a = 1.0 / g
        changes.append(np.linalg.norm(g - g_prev) / np.linalg.norm(g))
        g_prev = g
    em_tol = 1e-3
    # a threshold well away from every change value: the stop index is robust to rounding
    t_stop = next(i for i, c in enumerate(changes) if c < em_tol) + 1
    assert min(abs(np.log(np.array(changes) / em_tol))) > 0.05
    with CoFEM.dense(torch.eye(D, dtype=torch.float32, device="cuda"), torch.from_numpy(y).cuda(), beta, 4,
                     tol=1e-7, max_iter=50, seed=3) as gctx:
        st = gctx.em_run(60, em_tol)
    got = [x["gamma_change"] for x in st]
    _say("em_run on Phi = I: stopped after", len(st), "closed form", t_stop)
    assert len(st) == t_stop
    assert np.allclose(got, changes[:t_stop], rtol=1e-4)


def test_em_run_matches_oracle_stop(torch_dev):
    # a dense problem: GPU and oracle stop at the same EM iteration and report
    # the same relative changes (free-running trajectories, each with its own
    # CG stop decisions)
    torch = torch_dev
    p = synth.dense_256x1024(0)
    em_tol = 0.02
    with _ctx(torch, p) as g:
        st = g.em_run(p.T_em, em_tol)
        mu = g.posterior()[0].cpu().numpy()
    r = O.cofem(O.DenseOperator(p.phi.astype(np.float64)), p.y, p.beta, p.T_em, p.K, tol=p.tol,
                max_iter=p.max_iter, seed=p.seed, em_tol=em_tol)
    got = [x["gamma_change"] for x in st]
    ref = [x["gamma_change"] for x in r.stats]
    _say("em_run dense_256x1024: GPU", len(st), "oracle", len(r.stats), "changes", got[-3:], ref[-3:])
    assert len(st) == len(r.stats) < p.T_em
    assert np.allclose(got, ref, rtol=1e-3)
    assert relerr(mu, r.mu) < 1e-3


# ------------------------------------------------------------------ caller workspace
_WS_CASES = {
    "dense_fp32": (lambda: synth.dense_problem(300, 777, nnz=9, beta=5e3, K=13, tol=1e-6, seed=3), {}),
    "dense_bf16_ir_warm": (lambda: synth.dense_problem(200, 700, nnz=8, beta=1e3, K=12, tol=1e-5, seed=11),
                           {"precision": "bf16_ir", "warm_start": True}),
    "conv_warm_jacobi": (lambda: synth.conv_problem(40, 36, 5, rho=0.03, beta=1e3, K=8, tol=1e-5, seed=11),
                         {"warm_start": True, "jacobi": True}),
    "dct": (lambda: synth.dct_problem(4096, rho=0.04, beta=4e4, K=6, tol=1e-5, seed=2), {}),
}


@pytest.mark.parametrize("case", sorted(_WS_CASES))
def test_caller_workspace_is_bit_identical(torch_dev, case):
    # the same run with the library's own allocations and inside a torch
    # tensor sized by cofem_workspace_size: same bits, same CG counts
    torch = torch_dev
    mk, kw = _WS_CASES[case]
    p = mk()
    _say("workspace", case)
    outs = []
    for ws in (None, True):
        with _ctx(torch, p, workspace=ws, **kw) as g:
            if ws is True:
                assert g.workspace is not None and g.workspace.data_ptr() % 256 == 0
            st = g.em_step(3)
            X, m = g.solution()
            outs.append(([x["cg_iters"] for x in st], [x.cpu().numpy() for x in g.posterior()] +
                         [X.cpu().numpy(), m.cpu().numpy()]))
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)


def test_caller_workspace_batched_and_too_small(torch_dev):
    torch = torch_dev
    from paper_2202_12808_amd import cofem as C
    from paper_2202_12808_amd.cofem import CoFEMBatch
    rng = np.random.default_rng(4)
    pairs = []
    for D in (512, 1000):
        N = D // 4
        pairs.append((torch.from_numpy((rng.standard_normal((N, D)) / np.sqrt(N)).astype(np.float32)).cuda(),
                      torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()))
    res = []
    for ws in (None, True):
        with CoFEMBatch(pairs, 1e3, 8, tol=1e-5, seed=5, workspace=ws) as g:
            st = g.em_step(2)
            res.append(([[x["cg_iters"] for x in it] for it in st],
                        [t.cpu().numpy() for i in range(2) for t in g.posterior(i)]))
    assert res[0][0] == res[1][0]
    for a, b in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, b)
    # a workspace one byte short of the reported size is refused
    p = synth.dense_problem(64, 128, nnz=3, beta=100.0, K=4, tol=1e-6, seed=2)
    from paper_2202_12808_amd.cofem import CoFEM
    prob = C.cofem_problem(kind=C.COFEM_DENSE, N=64, D=128, phi=1, ld_phi=128, phi_dtype=C.COFEM_F32,
                           H=0, W=0, kh=0, kw=0, taps=None, y=2)
    params = CoFEM._params(p.beta, p.K, p.tol, p.max_iter, p.seed)
    n = C.cofem_workspace_size(prob, params)
    small = torch.empty(n - 1 + 256, dtype=torch.uint8, device="cuda")
    off = (-small.data_ptr()) % 256
    with pytest.raises(C.CofemError) as ei:
        CoFEM.dense(torch.from_numpy(p.phi).cuda(), torch.from_numpy(p.y).cuda(), p.beta, p.K, tol=p.tol,
                    workspace=small[off:off + n - 1])
    assert ei.value.status == C.COFEM_ERR_OUT_OF_MEMORY


# ------------------------------------------------------------------ several EM iterations per call
_PIPE_FORMS = {
    "dense_plain": (lambda: synth.dense_problem(200, 700, nnz=8, beta=1e3, K=12, tol=1e-5, seed=12), {}),
    "conv_plain_ragged": (lambda: synth.conv_problem(40, 36, 5, rho=0.03, beta=1e3, K=8, tol=1e-5, seed=12), {}),
    "conv_warm_jacobi": (lambda: synth.conv_problem(40, 36, 5, rho=0.03, beta=1e3, K=8, tol=1e-5, seed=12),
                         {"warm_start": True, "jacobi": True}),
    "conv_learned": (lambda: synth.conv_problem(64, 32, 5, rho=0.03, beta=1e3, K=8, tol=1e-5, seed=12),
                     {"spectral_start": True}),
    "dct_warm_jacobi": (lambda: synth.dct_problem(4096, rho=0.04, beta=4e4, K=6, tol=1e-5, seed=12),
                        {"warm_start": True, "jacobi": True}),
}


@pytest.mark.parametrize("form", sorted(_PIPE_FORMS))
def test_em_steps_in_one_call_equal_single_calls(torch_dev, form):
    # cofem_em_step(n) enqueues each EM iteration's start before it reads the
    # previous one's end; the device work is that of n calls of one
    # iteration: the same statistics (host clock aside), the same posterior
    # bits and the same timed launches
    torch = torch_dev
    from paper_2202_12808_amd.cofem import CoFEMNet
    mk, kw = _PIPE_FORMS[form]
    p = mk()
    _say("em_step(n) vs n x em_step(1)", form)
    net = CoFEMNet(p.H, p.W, seed=5) if form == "conv_learned" else None
    runs = []
    with _ctx(torch, p, **kw) as g:
        if net is not None:
            g.set_predictor(net)
        for one_by_one in (False, True):
            g.restart()
            g.set_kernel_timing(1)
            st = [g.em_step(1)[0] for _ in range(5)] if one_by_one else g.em_step(5)
            kt = g.kernel_timing()
            g.set_kernel_timing(0)
            runs.append((st, kt, [x.cpu().numpy() for x in g.posterior()], [x.cpu().numpy() for x in g.solution()]))
    if net is not None:
        net.close()
    (st_a, kt_a, post_a, sol_a), (st_b, kt_b, post_b, sol_b) = runs
    _say("cg", [x["cg_iters"] for x in st_a], [x["cg_iters"] for x in st_b])
    for a, b in zip(st_a, st_b):
        assert {k: v for k, v in a.items() if k != "ms"} == {k: v for k, v in b.items() if k != "ms"}
        assert a["ms"] > 0.0 and b["ms"] > 0.0
    assert {k: v[1] for k, v in kt_a.items()} == {k: v[1] for k, v in kt_b.items()}
    for a, b in zip(post_a + sol_a, post_b + sol_b):
        assert np.array_equal(a, b)
