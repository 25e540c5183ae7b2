"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This package builds matrices and right-hand sides only.  It holds none of the
preconditioner's arithmetic (no factorization, no solve, no Krylov step), so
both sides of every parity check can draw their inputs from it.
"""
from .generators import (  # noqa: F401
    CSR,
    splitmix64,
    uniform01,
    aniso5,
    aniso7,
    rotated9,
    convdiff5,
    slab_partition,
    block_partition,
    uniform_rhs,
    random_sparse,
    convdiff_batch_params,
    convdiff_batch,
    block_diagonal,
    workload,
)
from .serving import (  # noqa: F401
    Request,
    request_stream,
    build_matrix,
    general_sparse,
    arrival_times,
)
