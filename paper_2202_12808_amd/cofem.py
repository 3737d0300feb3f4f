"""ctypes binding of libcofem.so (declared in include/cofem.h).

Argument marshalling only: every step of the E-step and M-step runs in the
library's HIP kernels.  The functions keep the C names; tensors are torch
tensors on the GPU (PyTorch is used for device memory and streams), passed by
``data_ptr()``.  ``CoFEM`` bundles a context with the tensors it borrows.

Loading fails loudly (``CofemError``) when the library has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint64, c_void_p

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcofem.so")

COFEM_OK = 0
COFEM_ERR_INVALID_ARG = 1
COFEM_ERR_OUT_OF_MEMORY = 2
COFEM_ERR_DEVICE = 3
COFEM_ERR_NUMERIC = 4
COFEM_ERR_UNSUPPORTED = 5

COFEM_DENSE = 0
COFEM_CONV2D_CIRC = 1
COFEM_DCT_MASK = 2
COFEM_F32 = 0
COFEM_BF16 = 1
COFEM_PREC_FP32 = 0
COFEM_PREC_BF16_IR = 1
COFEM_PREC_FP64 = 2
COFEM_STOP_FROBENIUS = 0
COFEM_STOP_PER_COLUMN = 1
_STOP_RULES = {"frobenius": COFEM_STOP_FROBENIUS, "per_column": COFEM_STOP_PER_COLUMN}
COFEM_FLAG_TRUE_RESIDUAL = 1
COFEM_FLAG_EAGER = 2
COFEM_FLAG_BATCHED = 4
COFEM_FLAG_WARM_PREV = 8
COFEM_FLAG_JACOBI = 16
COFEM_FLAG_SPECTRAL_START = 32
_PRECISIONS = {"fp32": COFEM_PREC_FP32, "bf16_ir": COFEM_PREC_BF16_IR, "fp64": COFEM_PREC_FP64}
COFEM_MAX_K = 32


class CofemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_STATUS_NAMES = {0: "COFEM_OK", 1: "COFEM_ERR_INVALID_ARG", 2: "COFEM_ERR_OUT_OF_MEMORY",
                 3: "COFEM_ERR_DEVICE", 4: "COFEM_ERR_NUMERIC", 5: "COFEM_ERR_UNSUPPORTED"}


class cofem_problem(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("N", c_int64), ("D", c_int64), ("phi", c_void_p),
                ("ld_phi", c_int64), ("phi_dtype", c_int32), ("H", c_int32), ("W", c_int32),
                ("kh", c_int32), ("kw", c_int32), ("taps", c_void_p), ("y", c_void_p),
                ("rows", c_void_p), ("n_tasks", c_int32)]


class cofem_params(ctypes.Structure):
    _fields_ = [("beta", c_double), ("K", c_int32), ("cg_tol", c_double), ("cg_max_iter", c_int32),
                ("seed", c_uint64), ("precision", c_int32), ("stop_rule", c_int32),
                ("alpha_max", c_double), ("flags", c_int32), ("poll_interval", c_int32),
                ("ir_inner_tol", c_double), ("ir_max_sweeps", c_int32)]


class cofem_iter_stats(ctypes.Structure):
    _fields_ = [("t", c_int32), ("cg_iters", c_int32), ("converged", c_int32), ("n_clamped", c_int32),
                ("rel_resid", c_double), ("ms", c_double), ("rel_resid_true", c_double),
                ("ir_sweeps", c_int32), ("gamma_change", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_SIGNATURES = {
    "cofem_init": (c_int32, [POINTER(cofem_problem), c_int32, POINTER(cofem_params), c_void_p, c_void_p,
                             ctypes.c_size_t, POINTER(c_void_p)]),
    "cofem_workspace_size": (c_int32, [POINTER(cofem_problem), c_int32, POINTER(cofem_params),
                                       POINTER(ctypes.c_size_t)]),
    "cofem_em_step": (c_int32, [c_void_p, c_int32, POINTER(cofem_iter_stats)]),
    "cofem_em_run": (c_int32, [c_void_p, c_int32, c_double, POINTER(cofem_iter_stats), POINTER(c_int32)]),
    "cofem_em_step_static": (c_int32, [POINTER(cofem_problem), POINTER(cofem_params), c_void_p, c_int32, c_void_p,
                                       c_void_p, c_void_p, POINTER(cofem_iter_stats), c_void_p]),
    "cofem_posterior": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "cofem_set_alpha": (c_int32, [c_void_p, c_int32, c_void_p]),
    "cofem_set_iteration": (c_int32, [c_void_p, c_int32]),
    "cofem_restart": (c_int32, [c_void_p]),
    "cofem_set_fixed_cg_iters": (c_int32, [c_void_p, c_int32]),
    "cofem_get_solution": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "cofem_get_means": (c_int32, [c_void_p, c_int32, c_void_p]),
    "cofem_apply_A": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cofem_probe_signs": (c_int32, [c_uint64, c_int32, c_int32, c_int64, c_void_p, c_void_p]),
    "cofem_time_operator": (c_int32, [c_void_p, c_int32, POINTER(ctypes.c_float)]),
    "cofem_set_kernel_timing": (c_int32, [c_void_p, c_int32]),
    "cofem_net_num_params": (c_int64, []),
    "cofem_net_create": (c_int32, [c_int32, c_int32, c_uint64, c_void_p, POINTER(c_void_p)]),
    "cofem_net_destroy": (None, [c_void_p]),
    "cofem_net_set_params": (c_int32, [c_void_p, c_void_p, c_int64]),
    "cofem_net_get_params": (c_int32, [c_void_p, c_void_p, c_int64]),
    "cofem_net_forward": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "cofem_net_forward_bf16": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "cofem_net_loss_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double), c_void_p]),
    "cofem_net_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float, POINTER(c_double)]),
    "cofem_features": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "cofem_set_predictor": (c_int32, [c_void_p, c_void_p]),
    "cofem_batch_plan": (c_int32, [c_void_p, POINTER(c_int32), POINTER(ctypes.c_float), POINTER(c_int32),
                                   POINTER(c_int32)]),
    "cofem_get_ir_sweeps": (c_int32, [c_void_p, POINTER(c_int32), c_int32, POINTER(c_int32)]),
    "cofem_apply_A_lowp": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cofem_get_kernel_timing": (c_int32, [c_void_p, POINTER(ctypes.c_double), POINTER(c_int64)]),
    "cofem_kernel_name": (ctypes.c_char_p, [c_void_p, c_int32]),
    "cofem_destroy": (None, [c_void_p]),
    "cofem_last_error": (c_char_p, [c_void_p]),
    "cofem_status_string": (c_char_p, [c_int32]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libcofem.so (once) and declares every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise CofemError(COFEM_ERR_UNSUPPORTED,
                         f"{path} is missing: build it with `python -m paper_2202_12808_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != COFEM_OK:
        msg = load().cofem_last_error(ctx)
        raise CofemError(status, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


# --------------------------------------------------------- C-named wrappers
def cofem_workspace_size(problems, params: cofem_params) -> int:
    """Device bytes cofem_init needs for these problems (a list, or one)."""
    if isinstance(problems, cofem_problem):
        problems = [problems]
    arr = (cofem_problem * len(problems))(*problems)
    n = ctypes.c_size_t(0)
    _check(load().cofem_workspace_size(arr, len(problems), ctypes.byref(params), ctypes.byref(n)))
    return int(n.value)


def cofem_init(problem: cofem_problem, params: cofem_params, stream=None, workspace=None):
    """workspace: None (the library allocates) or a 256-byte aligned device
    tensor of at least cofem_workspace_size bytes, kept alive by the caller."""
    ctx = c_void_p()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().cofem_init(ctypes.byref(problem), 1, ctypes.byref(params), _stream(stream), _ptr(workspace),
                             nbytes, ctypes.byref(ctx)))
    return ctx


def cofem_em_step(ctx, n_iters: int, n_problems: int = 1):
    """Per-iteration statistics: a list of n_iters dicts, or for a batched
    context a list of n_iters lists of n_problems dicts."""
    stats = (cofem_iter_stats * max(n_iters * n_problems, 1))()
    _check(load().cofem_em_step(ctx, n_iters, stats), ctx)
    if n_problems == 1:
        return [stats[i].as_dict() for i in range(n_iters)]
    return [[stats[i * n_problems + j].as_dict() for j in range(n_problems)] for i in range(n_iters)]


def cofem_em_run(ctx, max_iters: int, em_tol: float, n_problems: int = 1):
    """EM iterations until the relative change of 1/alpha falls below em_tol
    (at most max_iters); statistics as cofem_em_step, one entry per iteration run."""
    stats = (cofem_iter_stats * max(max_iters * n_problems, 1))()
    n = c_int32(0)
    _check(load().cofem_em_run(ctx, max_iters, float(em_tol), stats, ctypes.byref(n)), ctx)
    if n_problems == 1:
        return [stats[i].as_dict() for i in range(n.value)]
    return [[stats[i * n_problems + j].as_dict() for j in range(n_problems)] for i in range(n.value)]


def cofem_em_step_static(problem: cofem_problem, params: cofem_params, alpha_in, t: int, mu=None, s=None,
                         alpha_out=None, stream=None):
    """One EM iteration without a context or any device allocation (the
    library's static scratch array); returns the iteration's statistics."""
    st = cofem_iter_stats()
    _check(load().cofem_em_step_static(ctypes.byref(problem), ctypes.byref(params), _ptr(alpha_in), int(t), _ptr(mu),
                                       _ptr(s), _ptr(alpha_out), ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def cofem_init_batch(problems, params: cofem_params, stream=None, workspace=None):
    arr = (cofem_problem * len(problems))(*problems)
    ctx = c_void_p()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(load().cofem_init(arr, len(problems), ctypes.byref(params), _stream(stream), _ptr(workspace), nbytes,
                             ctypes.byref(ctx)))
    return ctx


def cofem_batch_plan(ctx, n_problems: int):
    target = c_int32(0)
    ms = (ctypes.c_float * 4)()
    s1 = (c_int32 * n_problems)()
    s2 = (c_int32 * n_problems)()
    _check(load().cofem_batch_plan(ctx, ctypes.byref(target), ms, s1, s2), ctx)
    return {"target_wgs": target.value, "candidate_ms": [float(v) for v in ms],
            "splits1": list(s1), "splits2": list(s2)}


def cofem_posterior(ctx, mu=None, s=None, alpha=None, problem: int = 0):
    _check(load().cofem_posterior(ctx, problem, _ptr(mu), _ptr(s), _ptr(alpha)), ctx)


def cofem_set_alpha(ctx, alpha, problem: int = 0):
    _check(load().cofem_set_alpha(ctx, problem, _ptr(alpha)), ctx)


def cofem_set_iteration(ctx, t: int):
    _check(load().cofem_set_iteration(ctx, t), ctx)


def cofem_restart(ctx):
    _check(load().cofem_restart(ctx), ctx)


def cofem_set_fixed_cg_iters(ctx, n: int):
    _check(load().cofem_set_fixed_cg_iters(ctx, n), ctx)


def cofem_get_means(ctx, mu, problem: int = 0):
    _check(load().cofem_get_means(ctx, problem, _ptr(mu)), ctx)


def cofem_get_solution(ctx, probes=None, mean=None, problem: int = 0):
    _check(load().cofem_get_solution(ctx, problem, _ptr(probes), _ptr(mean)), ctx)


def cofem_apply_A(ctx, v_probes, v_mean, q_probes, q_mean, problem: int = 0):
    _check(load().cofem_apply_A(ctx, problem, _ptr(v_probes), _ptr(v_mean), _ptr(q_probes),
                                _ptr(q_mean)), ctx)


def cofem_apply_A_lowp(ctx, v_probes, v_mean, q_probes, q_mean, problem: int = 0):
    _check(load().cofem_apply_A_lowp(ctx, problem, _ptr(v_probes), _ptr(v_mean), _ptr(q_probes),
                                     _ptr(q_mean)), ctx)


def cofem_probe_signs(seed: int, t: int, K: int, D: int, out, stream=None):
    _check(load().cofem_probe_signs(seed, t, K, D, _ptr(out), _stream(stream)))


def cofem_time_operator(ctx, reps: int):
    out = (ctypes.c_float * 3)()
    _check(load().cofem_time_operator(ctx, reps, out), ctx)
    return [float(out[i]) for i in range(3)]


KERNEL_SLOTS = ("pass1", "pass2", "update", "init", "mstep", "check")  # COFEM_KT_* order


def cofem_get_ir_sweeps(ctx):
    counts = (c_int32 * 256)()
    n = c_int32(0)
    _check(load().cofem_get_ir_sweeps(ctx, counts, 256, ctx and ctypes.byref(n)), ctx)
    return [int(counts[i]) for i in range(min(n.value, 256))]


def cofem_set_kernel_timing(ctx, enable):
    """enable: False/0 off, True/1 every CG iteration, n > 1 every n-th."""
    _check(load().cofem_set_kernel_timing(ctx, int(enable)), ctx)


def cofem_kernel_name(ctx, slot: str):
    """The kernel a timing slot ("pass1", ...) times for this context."""
    name = load().cofem_kernel_name(ctx, KERNEL_SLOTS.index(slot))
    return name.decode() if name else None


def cofem_get_kernel_timing(ctx):
    """{slot: (total ms, launches)} since the last cofem_set_kernel_timing."""
    ms = (ctypes.c_double * len(KERNEL_SLOTS))()
    n = (c_int64 * len(KERNEL_SLOTS))()
    _check(load().cofem_get_kernel_timing(ctx, ms, n), ctx)
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_SLOTS)}


def cofem_destroy(ctx):
    if ctx:
        load().cofem_destroy(ctx)


# --------------------------------------------------------- convenience object
class CoFEM:
    """One CoFEM problem on the current GPU.

    dense:  CoFEM.dense(phi[N, D] float32 cuda, y[N] (or [T, N] for T tasks) float32 cuda, beta, K, ...)
    conv:   CoFEM.conv(taps[k, k] float32 cuda, y[H*W] (or [T, H*W] for T tasks) float32 cuda, H, W, beta, K, ...)
    dct:    CoFEM.dct(rows[N] int32 cuda, y[N] float32 cuda, D, beta, K, ...)
    """

    def __init__(self, problem: cofem_problem, params: cofem_params, keep, device, stream=None,
                 workspace=None):
        import torch
        self._keep = keep
        self.device = device
        self.D = int(problem.D)
        self.K = int(params.K)
        self.params = params
        self.problem = problem
        if workspace is True:
            # a caller-owned workspace from torch, sized by the library
            n = cofem_workspace_size(problem, params)
            workspace = torch.empty(n + 256, dtype=torch.uint8, device=device)
            off = (-workspace.data_ptr()) % 256
            workspace = workspace[off:off + n]
        self.workspace = workspace
        with torch.cuda.device(device):
            self.ctx = cofem_init(problem, params, stream, workspace)

    @staticmethod
    def _params(beta, K, tol, max_iter, seed, alpha_max=1e10, poll_interval=0, precision="fp32",
                true_residual=True, ir_inner_tol=0.0, ir_max_sweeps=0, warm_start=False, jacobi=False,
                stop_rule="frobenius", spectral_start=False):
        flags = ((COFEM_FLAG_TRUE_RESIDUAL if true_residual else 0) | (COFEM_FLAG_WARM_PREV if warm_start else 0)
                 | (COFEM_FLAG_JACOBI if jacobi else 0) | (COFEM_FLAG_SPECTRAL_START if spectral_start else 0))
        return cofem_params(beta=float(beta), K=int(K), cg_tol=float(tol), cg_max_iter=int(max_iter),
                            seed=int(seed) & 0xFFFFFFFFFFFFFFFF, precision=_PRECISIONS[precision],
                            stop_rule=_STOP_RULES[stop_rule], alpha_max=float(alpha_max), flags=flags,
                            poll_interval=int(poll_interval), ir_inner_tol=float(ir_inner_tol),
                            ir_max_sweeps=int(ir_max_sweeps))

    @classmethod
    def dense(cls, phi, y, beta, K, tol=1e-5, max_iter=400, seed=0, workspace=None, **kw):
        import torch
        if phi.dtype != torch.float32 or y.dtype != torch.float32 or not phi.is_cuda or not y.is_cuda:
            raise CofemError(COFEM_ERR_INVALID_ARG, "phi and y must be float32 GPU tensors")
        phi = phi.contiguous()
        y = y.contiguous()
        N, D = phi.shape
        T = 1 if y.dim() == 1 else int(y.shape[0])
        if y.numel() != T * N:
            raise CofemError(COFEM_ERR_INVALID_ARG, "y must be (N,) or (T, N)")
        prob = cofem_problem(kind=COFEM_DENSE, N=N, D=D, phi=phi.data_ptr(), ld_phi=D,
                             phi_dtype=COFEM_F32, H=0, W=0, kh=0, kw=0, taps=None, y=y.data_ptr(), n_tasks=T)
        ctx = cls(prob, cls._params(beta, K, tol, max_iter, seed, **kw), (phi, y), phi.device,
                  workspace=workspace)
        ctx.T = T
        return ctx

    @classmethod
    def conv(cls, taps, y, H, W, beta, K, tol=1e-5, max_iter=400, seed=0, workspace=None, **kw):
        import torch
        if taps.dtype != torch.float32 or y.dtype != torch.float32 or not taps.is_cuda or not y.is_cuda:
            raise CofemError(COFEM_ERR_INVALID_ARG, "taps and y must be float32 GPU tensors")
        taps = taps.contiguous()
        y = y.contiguous()
        th, tw = taps.shape
        T = 1 if y.dim() == 1 else int(y.shape[0])
        if y.numel() != T * H * W:
            raise CofemError(COFEM_ERR_INVALID_ARG, "y must be (H*W,) or (T, H*W)")
        prob = cofem_problem(kind=COFEM_CONV2D_CIRC, N=H * W, D=H * W, phi=None, ld_phi=0,
                             phi_dtype=COFEM_F32, H=H, W=W, kh=th, kw=tw, taps=taps.data_ptr(),
                             y=y.data_ptr(), n_tasks=T)
        ctx = cls(prob, cls._params(beta, K, tol, max_iter, seed, **kw), (taps, y), taps.device,
                  workspace=workspace)
        ctx.T = T
        return ctx

    @classmethod
    def dct(cls, rows, y, D, beta, K, tol=1e-5, max_iter=400, seed=0, workspace=None, **kw):
        """Inverse DCT of a length-D coefficient vector followed by the N
        observed samples `rows` (distinct indices into [0, D)).  y: (N,) for
        one task, or (T, N) for T tasks sharing alpha (multi-task SBL)."""
        import torch
        if rows.dtype != torch.int32 or y.dtype != torch.float32 or not rows.is_cuda or not y.is_cuda:
            raise CofemError(COFEM_ERR_INVALID_ARG, "rows must be an int32 and y a float32 GPU tensor")
        rows = rows.contiguous()
        y = y.contiguous()
        N = rows.numel()
        T = 1 if y.dim() == 1 else int(y.shape[0])
        if y.numel() != T * N:
            raise CofemError(COFEM_ERR_INVALID_ARG, "y must be (N,) or (T, N)")
        prob = cofem_problem(kind=COFEM_DCT_MASK, N=N, D=int(D), phi=None, ld_phi=0, phi_dtype=COFEM_F32,
                             H=0, W=0, kh=0, kw=0, taps=None, y=y.data_ptr(), rows=rows.data_ptr(), n_tasks=T)
        ctx = cls(prob, cls._params(beta, K, tol, max_iter, seed, **kw), (rows, y), rows.device,
                  workspace=workspace)
        ctx.T = T
        return ctx

    def em_step(self, n_iters=1):
        return cofem_em_step(self.ctx, n_iters)

    def em_run(self, max_iters, em_tol):
        """EM iterations until the relative change of 1/alpha is below em_tol."""
        return cofem_em_run(self.ctx, max_iters, em_tol)

    def posterior(self):
        import torch
        mu = torch.empty(self.D, dtype=torch.float32, device=self.device)
        s = torch.empty_like(mu)
        alpha = torch.empty_like(mu)
        cofem_posterior(self.ctx, mu, s, alpha)
        torch.cuda.synchronize(self.device)
        return mu, s, alpha

    def solution(self):
        import torch
        X = torch.empty((self.K, self.D), dtype=torch.float32, device=self.device)
        m = torch.empty(self.D, dtype=torch.float64, device=self.device)
        cofem_get_solution(self.ctx, X, m)
        torch.cuda.synchronize(self.device)
        return X, m

    def means(self):
        """(T, D) float64: every task's posterior mean after the last E-step."""
        import torch
        m = torch.empty((getattr(self, "T", 1), self.D), dtype=torch.float64, device=self.device)
        cofem_get_means(self.ctx, m)
        torch.cuda.synchronize(self.device)
        return m

    def set_alpha(self, alpha):
        alpha = alpha.to(device=self.device, dtype=self.dtype_f32()).contiguous()
        cofem_set_alpha(self.ctx, alpha)
        import torch
        torch.cuda.synchronize(self.device)

    @staticmethod
    def dtype_f32():
        import torch
        return torch.float32

    def set_iteration(self, t):
        cofem_set_iteration(self.ctx, t)

    def restart(self):
        """Algorithm 1 from its first line again: alpha = 1, t = 1, no previous solution."""
        cofem_restart(self.ctx)

    def set_fixed_cg_iters(self, n):
        cofem_set_fixed_cg_iters(self.ctx, n)

    def apply_A(self, v_probes, v_mean, lowp=False):
        """A v (or, with lowp, the bfloat16-dictionary operator of the
        mixed-precision form) for K probe columns (K x D) and the mean column."""
        import torch
        v_probes = v_probes.to(device=self.device, dtype=torch.float32).contiguous()
        v_mean = v_mean.to(device=self.device, dtype=torch.float64).contiguous()
        q = torch.empty_like(v_probes)
        qm = torch.empty_like(v_mean)
        (cofem_apply_A_lowp if lowp else cofem_apply_A)(self.ctx, v_probes, v_mean, q, qm)
        return q, qm

    def ir_sweeps(self):
        """Inner CG counts of the refinement sweeps of the last E-step."""
        return cofem_get_ir_sweeps(self.ctx)

    def time_operator(self, reps=20):
        return cofem_time_operator(self.ctx, reps)

    def features(self, net):
        """(feats [5, H*W], aux [3, H*W]) of the next E-step (convolution only)."""
        import torch
        feats = torch.empty((5, self.D), dtype=torch.float32, device=self.device)
        aux = torch.empty((3, self.D), dtype=torch.float32, device=self.device)
        _check(load().cofem_features(self.ctx, net.net, _ptr(feats), _ptr(aux)), self.ctx)
        return feats, aux

    def set_predictor(self, net):
        _check(load().cofem_set_predictor(self.ctx, net.net if net is not None else None), self.ctx)
        self._predictor = net

    def set_kernel_timing(self, enable=True):
        cofem_set_kernel_timing(self.ctx, enable)

    def kernel_timing(self):
        return cofem_get_kernel_timing(self.ctx)

    def kernel_name(self, slot):
        return cofem_kernel_name(self.ctx, slot)

    def close(self):
        if getattr(self, "ctx", None):
            cofem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class CoFEMBatch:
    """Many independent dense problems solved together (the batched form):
    bfloat16-rounded dictionaries, plain CG, grouped launches replayed from a
    captured graph.  problems: list of (phi[N_i, D_i] float32 cuda, y[N_i]
    float32 cuda); problem i uses probe seed `seed + i`."""

    def __init__(self, problems, beta, K, tol=1e-5, max_iter=400, seed=0, alpha_max=1e10, eager=False,
                 stream=None, workspace=None):
        import torch
        keep, probs = [], []
        for phi, y in problems:
            if phi.dtype != torch.float32 or y.dtype != torch.float32 or not phi.is_cuda or not y.is_cuda:
                raise CofemError(COFEM_ERR_INVALID_ARG, "phi and y must be float32 GPU tensors")
            phi, y = phi.contiguous(), y.contiguous()
            keep += [phi, y]
            N, D = phi.shape
            probs.append(cofem_problem(kind=COFEM_DENSE, N=N, D=D, phi=phi.data_ptr(), ld_phi=D,
                                       phi_dtype=COFEM_F32,
                                       H=0, W=0, kh=0, kw=0, taps=None, y=y.data_ptr()))
        self.n = len(probs)
        self.D = [int(p.D) for p in probs]
        self.K = int(K)
        self.device = problems[0][0].device
        self._keep = keep
        params = cofem_params(beta=float(beta), K=int(K), cg_tol=float(tol), cg_max_iter=int(max_iter),
                              seed=int(seed) & 0xFFFFFFFFFFFFFFFF, precision=COFEM_PREC_FP32,
                              stop_rule=COFEM_STOP_FROBENIUS, alpha_max=float(alpha_max),
                              flags=COFEM_FLAG_BATCHED | (COFEM_FLAG_EAGER if eager else 0), poll_interval=0,
                              ir_inner_tol=0.0,
                              ir_max_sweeps=0)
        if workspace is True:
            n = cofem_workspace_size(probs, params)
            workspace = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
            off = (-workspace.data_ptr()) % 256
            workspace = workspace[off:off + n]
        self.workspace = workspace
        with torch.cuda.device(self.device):
            self.ctx = cofem_init_batch(probs, params, stream, workspace)

    def em_step(self, n_iters=1):
        return cofem_em_step(self.ctx, n_iters, self.n)

    def em_run(self, max_iters, em_tol):
        return cofem_em_run(self.ctx, max_iters, em_tol, self.n)

    def posterior(self, i):
        import torch
        mu = torch.empty(self.D[i], dtype=torch.float32, device=self.device)
        s = torch.empty_like(mu)
        alpha = torch.empty_like(mu)
        cofem_posterior(self.ctx, mu, s, alpha, problem=i)
        torch.cuda.synchronize(self.device)
        return mu, s, alpha

    def set_alpha(self, i, alpha):
        import torch
        alpha = alpha.to(device=self.device, dtype=torch.float32).contiguous()
        cofem_set_alpha(self.ctx, alpha, problem=i)
        torch.cuda.synchronize(self.device)

    def set_iteration(self, t):
        cofem_set_iteration(self.ctx, t)

    def restart(self):
        cofem_restart(self.ctx)

    def solution(self, i):
        import torch
        X = torch.empty((self.K, self.D[i]), dtype=torch.float32, device=self.device)
        m = torch.empty(self.D[i], dtype=torch.float64, device=self.device)
        cofem_get_solution(self.ctx, X, m, problem=i)
        torch.cuda.synchronize(self.device)
        return X, m

    def plan(self):
        return cofem_batch_plan(self.ctx, self.n)

    def time_operator(self, reps=10):
        return cofem_time_operator(self.ctx, reps)

    def close(self):
        if getattr(self, "ctx", None):
            cofem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class CoFEMNet:
    """The learned form's network (convolution dictionaries): trained and run
    by the library's own kernels on H x W images."""

    def __init__(self, H, W, seed=0, stream=None):
        self.H, self.W = int(H), int(W)
        self.net = c_void_p()
        _check(load().cofem_net_create(self.H, self.W, int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream),
                                       ctypes.byref(self.net)))

    @staticmethod
    def num_params():
        return int(load().cofem_net_num_params())

    def set_params(self, theta):
        import numpy as np
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        _check(load().cofem_net_set_params(self.net, theta.ctypes.data_as(c_void_p), theta.size))

    def get_params(self):
        import numpy as np
        theta = np.empty(self.num_params(), dtype=np.float32)
        _check(load().cofem_net_get_params(self.net, theta.ctypes.data_as(c_void_p), theta.size))
        return theta

    def forward(self, feats):
        import torch
        out = torch.empty((2, self.H * self.W), dtype=torch.float32, device=feats.device)
        _check(load().cofem_net_forward(self.net, _ptr(feats.contiguous()), _ptr(out)))
        return out

    def forward_bf16(self, feats):
        """The predictor's forward pass (bfloat16 MFMA, float32 accumulation)."""
        import torch
        out = torch.empty((2, self.H * self.W), dtype=torch.float32, device=feats.device)
        _check(load().cofem_net_forward_bf16(self.net, _ptr(feats.contiguous()), _ptr(out)))
        return out

    def loss_grad(self, feats, aux, targets):
        import numpy as np
        loss = c_double(0.0)
        g = np.empty(self.num_params(), dtype=np.float32)
        _check(load().cofem_net_loss_grad(self.net, _ptr(feats.contiguous()), _ptr(aux.contiguous()),
                                          _ptr(targets.contiguous()), ctypes.byref(loss),
                                          g.ctypes.data_as(c_void_p)))
        return loss.value, g

    def train_step(self, feats, aux, targets, lr=1e-3):
        loss = c_double(0.0)
        _check(load().cofem_net_train_step(self.net, _ptr(feats), _ptr(aux), _ptr(targets), float(lr),
                                           ctypes.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "net", None) and self.net.value:
            load().cofem_net_destroy(self.net)
            self.net = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
