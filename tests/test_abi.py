"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/cofem.h, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re

import pytest

from paper_2202_12808_amd import cofem as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cofem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cofem_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(C.LIB_PATH):
        from paper_2202_12808_amd import build
        build.build()
    return C.load()


def test_header_declares_the_paper_entry_points():
    names = _declared()
    for n in ("cofem_init", "cofem_em_step", "cofem_posterior", "cofem_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(C._SIGNATURES)


def test_status_strings(lib):
    for code, name in C._STATUS_NAMES.items():
        assert lib.cofem_status_string(code).decode() == name


def _problem(**kw):
    p = C.cofem_problem(kind=C.COFEM_DENSE, N=8, D=16, phi=1, ld_phi=16, phi_dtype=C.COFEM_F32,
                        H=0, W=0, kh=0, kw=0, taps=None, y=2)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _params(**kw):
    q = C.cofem_params(beta=10.0, K=4, cg_tol=1e-5, cg_max_iter=100, seed=1, precision=0,
                       stop_rule=0, alpha_max=0.0, flags=0, poll_interval=0)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


@pytest.mark.parametrize("pkw,qkw,code", [
    ({}, {"beta": 0.0}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"beta": -1.0}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"K": 0}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"K": 33}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"cg_tol": -1.0}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"cg_max_iter": -1}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"precision": 7}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"precision": C.COFEM_PREC_BF16_IR, "ir_inner_tol": 1.5}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"precision": C.COFEM_PREC_BF16_IR, "ir_max_sweeps": -1}, C.COFEM_ERR_INVALID_ARG),
    ({"kind": C.COFEM_CONV2D_CIRC, "H": 4, "W": 4, "N": 16, "D": 16, "kh": 3, "kw": 3, "taps": 3},
     {"precision": C.COFEM_PREC_BF16_IR}, C.COFEM_ERR_UNSUPPORTED),
    ({}, {"precision": C.COFEM_PREC_FP64}, C.COFEM_ERR_UNSUPPORTED),
    ({}, {"stop_rule": 5}, C.COFEM_ERR_INVALID_ARG),
    ({}, {"precision": C.COFEM_PREC_BF16_IR, "stop_rule": C.COFEM_STOP_PER_COLUMN}, C.COFEM_ERR_UNSUPPORTED),
    ({"N": 0}, {}, C.COFEM_ERR_INVALID_ARG),
    ({"D": 0}, {}, C.COFEM_ERR_INVALID_ARG),
    ({"phi": None}, {}, C.COFEM_ERR_INVALID_ARG),
    ({"y": None}, {}, C.COFEM_ERR_INVALID_ARG),
    ({"ld_phi": 8}, {}, C.COFEM_ERR_INVALID_ARG),
    ({"kind": 9}, {}, C.COFEM_ERR_INVALID_ARG),
    ({"kind": C.COFEM_CONV2D_CIRC, "H": 4, "W": 4, "N": 16, "D": 16, "kh": 4, "kw": 4, "taps": 3}, {},
     C.COFEM_ERR_INVALID_ARG),
    ({"kind": C.COFEM_CONV2D_CIRC, "H": 4, "W": 4, "N": 16, "D": 16, "kh": 3, "kw": 5, "taps": 3}, {},
     C.COFEM_ERR_UNSUPPORTED),
    ({"kind": C.COFEM_CONV2D_CIRC, "H": 4, "W": 4, "N": 15, "D": 16, "kh": 3, "kw": 3, "taps": 3}, {},
     C.COFEM_ERR_INVALID_ARG),
    ({"kind": C.COFEM_CONV2D_CIRC, "H": 4, "W": 4, "N": 16, "D": 16, "kh": 3, "kw": 3, "taps": None}, {},
     C.COFEM_ERR_INVALID_ARG),
])
def test_init_rejects_bad_arguments_without_device(lib, pkw, qkw, code):
    ctx = ctypes.c_void_p()
    st = lib.cofem_init(ctypes.byref(_problem(**pkw)), 1, ctypes.byref(_params(**qkw)), None, None, 0,
                        ctypes.byref(ctx))
    assert st == code
    assert not ctx.value
    assert len(lib.cofem_last_error(None)) > 0


def test_init_rejects_batch_count(lib):
    ctx = ctypes.c_void_p()
    assert lib.cofem_init(ctypes.byref(_problem()), 0, ctypes.byref(_params()), None, None, 0,
                          ctypes.byref(ctx)) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_init(None, 1, ctypes.byref(_params()), None, None, 0,
                          ctypes.byref(ctx)) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_init(ctypes.byref(_problem()), 1, ctypes.byref(_params()), None, None, 0,
                          None) == C.COFEM_ERR_INVALID_ARG


def test_init_workspace_arguments_checked_first(lib):
    ctx = ctypes.c_void_p()
    # a misaligned workspace, and a size without a workspace, are rejected
    # before any device call
    assert lib.cofem_init(ctypes.byref(_problem()), 1, ctypes.byref(_params()), None, 8, 1 << 20,
                          ctypes.byref(ctx)) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_init(ctypes.byref(_problem()), 1, ctypes.byref(_params()), None, None, 1 << 20,
                          ctypes.byref(ctx)) == C.COFEM_ERR_INVALID_ARG
    assert not ctx.value


def _ws(lib, prob, params, n=1):
    arr = (C.cofem_problem * n)(*([prob] * n))
    nbytes = ctypes.c_size_t(0)
    st = lib.cofem_workspace_size(arr, n, ctypes.byref(params), ctypes.byref(nbytes))
    return st, nbytes.value


def test_workspace_size_without_device(lib):
    # the sizing pass touches no device and no device pointer (phi and y are
    # dummies here): dense needs at least the two packed float32 copies of Phi
    # (N and D padded to multiples of 64) and the four D x 32 CG blocks
    st, n1 = _ws(lib, _problem(N=100, D=300, ld_phi=300), _params())
    assert st == C.COFEM_OK
    Np, Dp = 128, 320
    assert n1 >= 2 * 4 * Np * Dp + 4 * 4 * Dp * 32
    st, n2 = _ws(lib, _problem(N=200, D=600, ld_phi=600), _params())
    assert st == C.COFEM_OK and n2 > n1
    # the mixed-precision form adds the two bfloat16 copies and the accumulated solution
    st, n3 = _ws(lib, _problem(N=100, D=300, ld_phi=300), _params(precision=C.COFEM_PREC_BF16_IR))
    assert st == C.COFEM_OK and n3 >= n1 + 2 * 2 * Np * Dp
    # conv: K + 1 columns of images (float32 probes, float64 mean), several blocks
    conv = _problem(kind=C.COFEM_CONV2D_CIRC, H=64, W=48, N=64 * 48, D=64 * 48, kh=7, kw=7, taps=3, phi=None)
    st, nc = _ws(lib, conv, _params(K=8))
    assert st == C.COFEM_OK and nc >= 4 * (4 * 8 + 8) * 64 * 48
    # batched: more problems need more memory; bad arguments are still rejected
    st, nb1 = _ws(lib, _problem(N=100, D=300, ld_phi=300), _params(), 2)
    st2, nb2 = _ws(lib, _problem(N=100, D=300, ld_phi=300), _params(), 4)
    assert st == st2 == C.COFEM_OK and nb2 > nb1
    assert _ws(lib, _problem(), _params(beta=-1.0))[0] == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_workspace_size(ctypes.byref(_problem()), 1, ctypes.byref(_params()), None) == \
        C.COFEM_ERR_INVALID_ARG


def test_spectral_start_sizing_and_rejections(lib):
    # the spectral start adds its transform workspace (ceil((K + 1)/2) complex
    # float32 images), the |h_hat|^2 table and the twiddles; it needs a single
    # convolution problem with power-of-two sides up to 4096
    conv = dict(kind=C.COFEM_CONV2D_CIRC, H=64, W=128, N=64 * 128, D=64 * 128, kh=7, kw=7, taps=3, phi=None)
    st0, n0 = _ws(lib, _problem(**conv), _params(K=7))
    st1, n1 = _ws(lib, _problem(**conv), _params(K=7, flags=C.COFEM_FLAG_SPECTRAL_START))
    D = 64 * 128
    assert st0 == st1 == C.COFEM_OK
    assert n1 - n0 >= 4 * D * 8 + D * 4 + 64 * 8
    assert n1 - n0 <= 4 * D * 8 + D * 4 + 64 * 8 + 3 * 256
    flag = _params(flags=C.COFEM_FLAG_SPECTRAL_START)
    for bad in (dict(conv, H=48, N=48 * 128, D=48 * 128), dict(conv, W=8192, N=64 * 8192, D=64 * 8192)):
        assert _ws(lib, _problem(**bad), flag)[0] == C.COFEM_ERR_UNSUPPORTED
        assert b"power-of-two" in lib.cofem_last_error(None)
    assert _ws(lib, _problem(), flag)[0] == C.COFEM_ERR_UNSUPPORTED
    dct = _problem(kind=C.COFEM_DCT_MASK, N=8, D=16, phi=None, ld_phi=0, rows=4)
    assert _ws(lib, dct, flag)[0] == C.COFEM_ERR_UNSUPPORTED
    # the allocation-free step takes any alpha: it has no spectral start
    st = lib.cofem_em_step_static(ctypes.byref(_problem(**conv)), ctypes.byref(flag), 5, 1, None, None, None,
                                  None, None)
    assert st == C.COFEM_ERR_UNSUPPORTED


def test_null_context_calls_fail_cleanly(lib):
    assert lib.cofem_em_step(None, 1, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_em_run(None, 1, 0.0, None, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_restart(None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_posterior(None, 0, None, None, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_set_alpha(None, 0, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_set_iteration(None, 1) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_set_fixed_cg_iters(None, 1) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_get_solution(None, 0, None, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_apply_A(None, 0, None, None, None, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_probe_signs(0, 1, 1, 10, None, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_probe_signs(0, -1, 1, 10, 8, None) == C.COFEM_ERR_INVALID_ARG
    assert lib.cofem_kernel_name(None, 0) is None
    lib.cofem_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(C.CofemError):
        C._lib_saved = C._lib
        try:
            C._lib = None
            C.load(str(tmp_path / "missing.so"))
        finally:
            C._lib = C._lib_saved
