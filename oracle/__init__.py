"""CPU oracle (test infrastructure only; see naj_oracle's module docstring)."""
from .naj_oracle import (  # noqa: F401
    STATUS_BREAKDOWN, STATUS_NOT_CONVERGED, STATUS_OK, MixedResult, OracleResult,
    accelerated_jacobi, accelerated_jacobi_mixed, alpha_next, block_apply_fp32, block_jacobi_blocks,
    block_matrix, block_solve, csr, dense_limit_spsd, dense_solution_spd, fused_step, inner_solve_fp32,
    jacobi_diagonal, objective, sdd_scalar_run,
)
