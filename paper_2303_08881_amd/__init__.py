"""Python binding of libschurilu (argument marshalling only).

Every numerical step runs in the gfx950 HIP kernels behind the C ABI declared
in include/schurilu.h; PyTorch supplies device memory and the current stream.
Importing this package does not load the library; the first call does, and it
raises if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    BJ,
    SCHUR,
    RAP,
    ILU0,
    MILU0,
    ILUT,
    PIVOT_ERROR,
    PIVOT_PERTURB,
    TRSV_AUTO,
    TRSV_LEVELS,
    TRSV_BLOCK,
    PREC_F64,
    PREC_F32,
    PREC_F16,
    ARNOLDI_AUTO,
    ARNOLDI_PER_PASS,
    OK,
    NOT_CONVERGED,
    SchurILUError,
    DeviceCSR,
    Precond,
    setup,
    fgmres,
    spmv,
    Batch,
    batch_setup,
    Server,
    memory_trim,
    lib,
    LIB_PATH,
    EXPORT,
    KERNEL_ALL,
)
