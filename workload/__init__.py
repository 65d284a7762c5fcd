"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package generates *inputs* only: a random mass-action mechanism, its
shared Jacobian sparsity pattern, and per-cell Jacobian values, step sizes and
right-hand sides.  It holds none of the solver's arithmetic (forming
``I - gamma*J``, BiCGStab, LU, adjoints): those live, independently, in the
oracle and in the HIP library.

The paper's workload (CB05 + isoprene SOA, 156 species, Section 4.2) is not
available; these mechanisms stand in for it with the same structure: a stiff,
sparse chemical Jacobian shared by every grid cell, values differing per cell
(the "realistic" case of Section 4.2) or identical in every cell (the "ideal"
case).
"""
from .mechanism import (  # noqa: F401
    Mechanism,
    gen_mechanism,
    rates,
    jacobian_values,
    gen_cells,
    config_inputs,
    CONFIGS,
    mech_seed,
    cell_seed,
)
