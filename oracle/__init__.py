"""FP64 CPU oracle for the CoFEM E-step hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
HIP product path never calls it, and this package imports nothing from the
HIP package: the two share no code, table or constant generator.
"""
from .cofem_oracle import (  # noqa: F401
    ALPHA_MAX_DEFAULT,
    ConvOperator,
    ConvOperatorFFT,
    DctMaskOperator,
    DenseOperator,
    cg_solve,
    cofem,
    cofem_estep,
    cofem_estep_ir,
    cofem_estep_pcg,
    diag_estimate,
    diag_estimate_ratio,
    exact_estep,
    exact_em,
    gamma_change,
    ir_solve,
    loglik,
    loglik_direct,
    make_apply_A,
    mstep,
    pcg_solve,
    rademacher_probes,
    spectral_operator,
    splitmix64_mix,
    splitmix64_stream,
    true_relative_residual,
)
