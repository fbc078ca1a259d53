"""Seeded synthetic inputs for the PPCG solver and its oracle.

This module only builds inputs: sparse SPD matrices in CSR form, exact
solutions and right-hand sides.  It holds none of the solver's arithmetic and
is shared, unchanged, by the HIP path's tests and benchmark and by the CPU
oracle's tests.
"""

from .gen import (  # noqa: F401
    CSR,
    poisson2d,
    poisson3d,
    poisson125,
    stencil27_lognormal,
    random_spd,
    shifted,
    rhs_from_solution,
    xstar_uniform,
    xstar_paper,
    poisson2d_eigpair,
    poisson3d_eigpair,
    batch_c4,
    nnz_poisson2d,
    nnz_poisson3d,
    nnz_stencil27,
    nnz_poisson125,
)
