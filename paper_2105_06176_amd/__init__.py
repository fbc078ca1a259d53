"""MI355X (gfx950) Pipelined PCG library: HIP kernels behind a C ABI.

``ppcg`` is the ctypes binding of ``libppcg.so`` (see ``include/ppcg.h``);
``build`` compiles the library in-tree with hipcc.
"""

from .ppcg import (  # noqa: F401
    BREAKDOWN, ERR_BAD_CSR, ERR_BUDGET, ERR_INVALID_ARG, NOT_CONVERGED, OK, STAGNATED,
    Hybrid, PPCGError, Server, Shard, Solver, footprint_bytes, lib, make_options, solve_batch, split_rows,
)
