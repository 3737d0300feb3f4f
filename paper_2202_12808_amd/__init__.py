"""MI355X-native CoFEM E-step hot path (covariance-free EM for sparse Bayesian
learning, arXiv 2202.12808).

The compute lives in ``libcofem.so`` (hand-written HIP for gfx950) behind the C
ABI declared in ``include/cofem.h``; ``paper_2202_12808_amd.cofem`` is a thin
ctypes binding with the same names.  Nothing is loaded at import time, so the
input generators in ``paper_2202_12808_amd.synth`` work on machines without a GPU.
"""
__all__ = ["cofem", "synth"]
