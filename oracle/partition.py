"""Performance model and 2-D data decomposition (Hybrid-PIPECG-3, Section IV-C
of Tiwari & Vadhiyar) -- plain reference for the row-split planner and the
split SpMV.

TEST INFRASTRUCTURE ONLY.  Only the tests may import this module; it shares
no code with the HIP library.

What it computes, following the subsections "Performance Modelling" and
"Data Decomposition" of Section IV-C:

* relative_performance: every processing unit k runs the same SpMV over all
  nnz entries in time t_k; its speed is s_k = nnz / t_k and its relative
  performance r_k = s_k / sum_j s_j.
* split_rows: unit k is given a share nnz_k = nnz * r_k of the non-zeros, but
  whole rows are assigned: the rows of the first unit are the most leading
  rows whose non-zeros number at most nnz_1 (equal to or slightly less).  The
  paper has two units (CPU first, then GPU, which takes the rest); for more
  units the same rule is applied to the cumulative shares, so that unit k
  ends at the most leading rows holding at most nnz * (r_1 + ... + r_k)
  non-zeros, and the last unit takes the rest.  With two units this is the
  paper's rule exactly.
* decompose: for the rows [lo, hi) of one unit, the entries whose column is
  also in [lo, hi) (nnz1: they need only the unit's own part of the vector)
  and the rest (nnz2: they need the elements owned by the other units, which
  have to be copied in first), and the sorted list of those remote columns.
* split_spmv: y = A x for the rows [lo, hi) computed as the paper's SpMV part 1
  over the nnz1 entries plus part 2 over the nnz2 entries, each part summed in
  the stored column order, and y_i = part1_i + part2_i.
"""

import numpy as np


def relative_performance(nnz, times):
    """r_k = s_k / sum_j s_j with s_k = nnz / t_k."""
    s = [nnz / float(t) for t in times]
    tot = sum(s)
    return [sk / tot for sk in s]


def rows_within(rp, nnz_target):
    """Most leading rows whose non-zeros number at most nnz_target."""
    rp = np.asarray(rp)
    k = 0
    while k < len(rp) - 1 and rp[k + 1] <= nnz_target:
        k += 1
    return k


def split_rows(rp, times):
    """Row boundaries [0, b_1, ..., b_K = n] for K units with the given SpMV times."""
    rp = np.asarray(rp)
    n = len(rp) - 1
    nnz = int(rp[-1])
    r = relative_performance(nnz, times)
    bounds = [0]
    cum = 0.0
    for k in range(len(times) - 1):
        cum += r[k]
        b = rows_within(rp, nnz * cum)
        bounds.append(max(b, bounds[-1]))
    bounds.append(n)
    return bounds


def decompose(rp, ci, lo, hi):
    """(nnz1, nnz2, remote columns) of the rows [lo, hi)."""
    nnz1 = nnz2 = 0
    remote = set()
    for i in range(lo, hi):
        for k in range(rp[i], rp[i + 1]):
            c = int(ci[k])
            if lo <= c < hi:
                nnz1 += 1
            else:
                nnz2 += 1
                remote.add(c)
    return nnz1, nnz2, sorted(remote)


def split_spmv(rp, ci, val, x, lo, hi):
    """Part 1 (local columns) + part 2 (remote columns) for the rows [lo, hi)."""
    y = np.zeros(hi - lo)
    for i in range(lo, hi):
        p1 = 0.0
        p2 = 0.0
        for k in range(rp[i], rp[i + 1]):
            c = int(ci[k])
            prod = val[k] * x[c]
            if lo <= c < hi:
                p1 = p1 + prod
            else:
                p2 = p2 + prod
        y[i - lo] = p1 + p2
    return y
