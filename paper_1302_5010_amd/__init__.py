"""Batch-mode Matching Pursuit LASSO (BMPL) on AMD MI355X.

A thin ctypes binding over ``libbmpl.so`` (the C ABI in ``include/bmpl.h``).
Every step of the solver runs in the library's HIP kernels; this module only
marshals device pointers, sizes and streams.  PyTorch provides device memory
and streams.  There is no CPU fallback: if the library is missing the import
of :mod:`paper_1302_5010_amd._binding` raises.

Layouts: the dictionary is passed atom-major as ``At`` (m, n) float32, which
is the column-major n x m matrix A with leading dimension n; signals as ``Bt``
(p, n) float32, one signal per row (column-major B).
"""
from ._binding import (  # noqa: F401
    BMPL_SIG_CAP_ACTIVE,
    BMPL_SIG_CAP_ITERS,
    BMPL_SIG_CONVERGED,
    BMPL_SIG_EARLY,
    BMPL_SIG_FALLBACK,
    BMPL_SIG_INEXACT,
    BMPL_SIG_NONFINITE,
    BmplError,
    ProposalNet,
    Solver,
    library_path,
    mlp_param_count,
    topk,
)
