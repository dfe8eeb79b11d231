"""FP64 CPU oracle for the PERF Gauss-Newton / PCG path.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports it, and it
imports nothing from the product package.

The per-ray work (tracing, partials, gradient rows, J products, blocks) is in
plain C (`perf_oracle.c`, built with gcc, OpenMP over rays, double precision).
The solver layer (preconditioner inverses, PCG of Alg. 2, the backtracking of
Alg. 3 and the Gauss-Newton update of Eq. 7) is plain numpy in float64 here.
"""
from .core import (  # noqa: F401
    OracleScene,
    build_oracle,
    library_path,
    jacobi_diag,
    jacobi_inverse,
    block_matrix,
    block_inverse,
    apply_block_inverse,
    apply_precond,
    pcg,
    line_search,
    project,
    gn_step,
    upsample,
    psnr,
    PCGResult,
)
