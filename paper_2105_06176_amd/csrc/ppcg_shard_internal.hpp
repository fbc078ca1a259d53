// ppcg_shard_internal.hpp -- one unit's share of A under the 2-D
// decomposition (Section IV-C), shared by the shard ABI and the host + GPU
// execution.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "ppcg_engine.hpp"

struct ppcg_shard {
    int device = 0;
    hipStream_t stream = nullptr;
    int n = 0, lo = 0, hi = 0;
    int64_t nnz1 = 0, nnz2 = 0;
    int halo = 0, nb = 0;
    int nch1 = 0, nch2 = 0;
    std::vector<int> halo_cols;  // host copy
    ppcg::DevArena arena;
    int64_t *cptr1 = nullptr, *cptr2 = nullptr;
    int *col1 = nullptr, *col2 = nullptr, *brow = nullptr, *hcols = nullptr;
    double *val1 = nullptr, *val2 = nullptr;
};

// Launch part 1 (which = 1: y = A_local x_local) or part 2 (which = 2:
// y += A_remote x_halo) of the shard's SpMV on its stream; e0/e1 may be NULL.
ppcg_status shard_launch(ppcg_shard *s, int which, const double *x_local, const double *x_halo,
                         double *y, hipEvent_t e0, hipEvent_t e1);
