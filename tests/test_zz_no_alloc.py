"""The allocation-free entry point cofem_em_step_static against the
context-based path (cofem_init, cofem_set_alpha, cofem_set_iteration,
cofem_em_step, cofem_posterior) on the same inputs: the same kernels run on
memory laid out in the library's static array, so the results must be the
same bits.  Two calls in a row, the second on a smaller problem, check that
the shared array is rebuilt and cleared between calls."""
import sys

import numpy as np
import pytest

from paper_2202_12808_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


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


def _both(torch, p, t, alpha, **kw):
    """(context path, static path): stats and (mu, s, alpha) of one EM step."""
    from paper_2202_12808_amd import cofem as C
    a_in = torch.from_numpy(alpha.astype(np.float32)).cuda()
    with _ctx(torch, p, **kw) as g:
        g.set_alpha(a_in)
        g.set_iteration(t)
        st_ref = g.em_step(1)[0]
        ref = [x.cpu().numpy() for x in g.posterior()]
        problem, params = g.problem, g.params
        keep = g._keep  # the caller's Phi / taps / rows and y stay alive for the static call
        mu = torch.empty(p.D, dtype=torch.float32, device="cuda")
        s = torch.empty_like(mu)
        a_out = torch.empty_like(mu)
        st = C.cofem_em_step_static(problem, params, a_in, t, mu, s, a_out)
        got = [x.cpu().numpy() for x in (mu, s, a_out)]
        del keep
    return st_ref, ref, st, got


_SEQUENCES = {
    "dense": [synth.dense_problem(300, 777, nnz=9, beta=5e3, K=13, tol=1e-6, seed=3),
              synth.dense_problem(128, 256, nnz=4, beta=1e3, K=7, tol=1e-6, seed=5)],
    "conv": [synth.conv_problem(72, 60, 7, rho=0.02, beta=100.0, K=8, tol=1e-6, seed=1, law="laplace"),
             synth.conv_problem(40, 36, 5, rho=0.03, beta=1e3, K=4, tol=1e-5, seed=2)],
    "dct": [synth.dct_problem(8192, rho=0.04, beta=4e4, K=9, tol=1e-5, seed=2),
            synth.dct_problem(4096, rho=0.04, beta=4e4, K=5, tol=1e-5, seed=4)],
}


@pytest.mark.parametrize("kind", sorted(_SEQUENCES))
def test_static_step_equals_context_step(torch_dev, kind):
    torch = torch_dev
    rng = np.random.default_rng(17)
    kw = {"jacobi": True} if kind != "dense" else {}
    for i, p in enumerate(_SEQUENCES[kind]):
        # a non-trivial alpha (as after a few M-steps) and a later probe draw
        alpha = 10.0 ** rng.uniform(-1.0, 3.0, p.D)
        t = 3 + i
        _say("static step", kind, "call", i, "D", p.D, "K", p.K)
        st_ref, ref, st, got = _both(torch, p, t, alpha, **kw)
        assert st["t"] == st_ref["t"] == t
        assert st["cg_iters"] == st_ref["cg_iters"] and st["converged"] == st_ref["converged"]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_static_step_rejects_what_it_cannot_hold(torch_dev):
    torch = torch_dev
    from paper_2202_12808_amd import cofem as C
    from paper_2202_12808_amd.cofem import CoFEM
    # 4096 x 16384 needs two packed float32 copies of Phi (512 MiB): beyond the 64 MiB array
    prob = C.cofem_problem(kind=C.COFEM_DENSE, N=4096, D=16384, phi=1, ld_phi=16384, phi_dtype=C.COFEM_F32,
                           H=0, W=0, kh=0, kw=0, taps=None, y=2)
    params = CoFEM._params(1e3, 32, 1e-5, 400, 0)
    a = torch.ones(16384, dtype=torch.float32, device="cuda")
    with pytest.raises(C.CofemError) as ei:
        C.cofem_em_step_static(prob, params, a, 1)
    assert ei.value.status == C.COFEM_ERR_INVALID_ARG
    with pytest.raises(C.CofemError) as ei:
        C.cofem_em_step_static(prob, CoFEM._params(1e3, 32, 1e-5, 400, 0, warm_start=True), a, 1)
    assert ei.value.status == C.COFEM_ERR_UNSUPPORTED
