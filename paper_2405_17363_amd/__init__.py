"""Batched Block-cells BiCGStab for (I - gamma*J) x = b on AMD gfx950.

Thin Python binding over the C-ABI library ``libbcs.so`` (include/bcs.h).
Every step of a solve runs in the library's HIP kernels; this module only
marshals torch tensors (device memory) and the current HIP stream.  There is
no fallback: if the library is missing or fails to load, the import of the
entry points raises.

    plan = Plan(row_ptr, col_idx, precond="jacobi")          # shared pattern ("ilu0": ILU(0))
    x, iters, resid, status, _ = solve_batch(plan, J, gamma, b)  # per-cell values
    x, status = BatchedSolve.apply(J, gamma, b, plan)            # differentiable
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    BCS_A_DIRECT,
    BCS_BREAKDOWN,
    BCS_BUDGET_CELL,
    BCS_BUDGET_INNER,
    BCS_CONVERGED,
    BCS_FP32_REFINE,
    BCS_FP64,
    BCS_GRAD_A,
    BCS_GRAD_VALUES,
    BCS_J_GAMMA,
    BCS_MAXIT,
    BCS_NONFINITE,
    BCS_PART_A,
    BCS_PART_AT,
    BCS_PART_LOWER,
    BCS_PART_UPPER,
    BCS_PRECOND_ILU0,
    BCS_PRECOND_JACOBI,
    BCS_PRECOND_NONE,
    BCS_SCHED_DIAG,
    BCS_SCHED_SPAN,
    NOALLOC_MAX_BYTES,
    NOALLOC_MAX_CELLS,
    BcsError,
    BatchedSolve,
    BatchedSolveWarning,
    Mechanism,
    Plan,
    assemble,
    exported_symbols,
    ilu_describe,
    lib,
    library_path,
    multi_autotune,
    schedule_describe,
    solve_batch,
    solve_batch_adjoint,
    solve_batch_mech,
    solve_batch_noalloc,
    solve_multi,
)
