"""SELL on chunk-shared offset lists (PPCG_FLAG_SELL_SHARED_OFFSETS).

When the column offsets (column minus row) of the 64 rows of each chunk,
merged, form one list (the chunk then stores that many slots: its longest row
or, where rows of different kinds meet, a few more), the rows are stored on
that list, with explicit zeros where a row lacks an offset, and the FP64
PIPECG SpMV reads the list instead of a column per entry.  Each row keeps its
entries in ascending column order with exact zeros between them, so:

* the SpMV equals the oracle's bit for bit (finite inputs: adding a zero
  product to a sum started at +0 changes nothing);
* iterates equal those of the per-entry-column storage bit for bit, in both
  iteration forms, alone and batched, and meet the 1e-10 bar against the
  oracle.

Whether a matrix qualifies is decided on the device; `shared_eligible`
states the rule independently on the host from the CSR arrays.
"""

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Solver, solve_batch
from shared_rule import shared_eligible
from workloads import (poisson125, poisson2d, poisson3d, random_spd, rhs_from_solution, shifted,
                       stencil27_lognormal, xstar_uniform)

pytestmark = pytest.mark.gpu

SH = ppcg.FLAG_SELL_SHARED_OFFSETS
NOSH = ppcg.FLAG_SELL_NO_SHARED_OFFSETS
VT = ppcg.FLAG_SELL_VALUE_TABLE
FV = ppcg.FLAG_SELL_FULL_VALUES
FUSED = ppcg.FLAG_ITER_FUSED
TWO = ppcg.FLAG_ITER_TWO_LAUNCH


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


MATS = {
    "poisson2d_2": lambda: poisson2d(2),          # 4 rows, offsets -2..2 in rows of 3: no list
    "poisson2d_37_ragged": lambda: poisson2d(37),  # chunks straddle grid lines
    "poisson2d_64": lambda: poisson2d(64),
    "poisson3d_24": lambda: poisson3d(24),
    "poisson3d_40": lambda: poisson3d(40),
    "stencil27_12": lambda: stencil27_lognormal(12, seed=3),
    "stencil27_20": lambda: stencil27_lognormal(20, seed=3),
    "poisson125_12": lambda: poisson125(12),
    "stencil27_40": lambda: stencil27_lognormal(40, seed=3),   # rows in their own order
    "poisson125_40": lambda: poisson125(40),
    "shifted_poisson2d_46": lambda: shifted(poisson2d(46), 0.1),
    "random_spd_3001": lambda: random_spd(3001, seed=2),  # random columns: never
}


# stencils whose rows SELL keeps in their own order (little padding) and
# that have shared lists: the SpMV above must run on them
SHARED_EXPECTED = {"poisson2d_37_ragged", "poisson2d_64", "poisson3d_24", "poisson3d_40", "stencil27_40",
                   "poisson125_40", "shifted_poisson2d_46"}


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("vflag", [VT, FV])
def test_spmv_on_shared_lists_is_bitwise(name, vflag):
    A = MATS[name]()
    S = Solver(A, spmv_format="sell", flags=SH | vflag)
    mi = S.matrix_info()
    expect = mi["sell_sigma"] == 1 and shared_eligible(A)
    print(f"{name}: sigma {mi['sell_sigma']} eligible {expect} col_index_bytes {mi['col_index_bytes']}")
    assert (mi["col_index_bytes"] == 0) == expect, name
    if name in SHARED_EXPECTED:
        assert expect, name
    for seed in (7, 8):
        x = xstar_uniform(A.n, seed)
        assert np.array_equal(host(S.spmv(dev(x))), oracle.spmv(A, x)), (name, seed)
    S.close()


def test_flags_refused_together_and_switch_off():
    A = poisson3d(24)
    with pytest.raises(ppcg.PPCGError):
        Solver(A, flags=SH | NOSH)
    assert Solver(A, spmv_format="sell", flags=NOSH).matrix_info()["col_index_bytes"] in (2, 4)
    # a pinned column layout keeps per-entry columns unless the lists are forced
    assert Solver(A, spmv_format="sell", flags=ppcg.FLAG_SELL_COL16).matrix_info()["col_index_bytes"] == 2
    assert Solver(A, spmv_format="sell", flags=ppcg.FLAG_SELL_COL32 | SH).matrix_info()["col_index_bytes"] == 0


ITER_CASES = {
    # generator, fixed iteration counts
    "poisson3d_40": (lambda: poisson3d(40), (25, 100)),
    "poisson2d_100_ragged": (lambda: poisson2d(100), (3, 40)),
    # (rows in their own order: SELL sorts the rows of smaller 27- and
    # 125-point grids, whose boundary rows are short)
    "stencil27_40": (lambda: stencil27_lognormal(40, seed=3), (10, 20)),
    "poisson125_40": (lambda: poisson125(40), (5, 15)),
    # 360,000 rows: 3 rows per thread in the single launch, ragged last tile
    "poisson2d_600_three_rows": (lambda: poisson2d(600), (4, 45)),
    # 1,906,624 rows: 5 rows per thread
    "poisson3d_124_five_rows": (lambda: poisson3d(124), (3, 12)),
}


@pytest.mark.parametrize("name", sorted(ITER_CASES))
@pytest.mark.parametrize("form", [FUSED, TWO])
def test_fixed_iterates_equal_per_entry_columns_and_oracle(name, form):
    gen, ks = ITER_CASES[name]
    A = gen()
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    S = Solver(A, fixed_iters=1, spmv_format="sell", flags=SH | form)
    N = Solver(A, fixed_iters=1, spmv_format="sell", flags=NOSH | form)
    assert S.matrix_info()["col_index_bytes"] == 0
    assert N.matrix_info()["col_index_bytes"] in (2, 4)
    assert S.matrix_info()["bytes_spmv"] < N.matrix_info()["bytes_spmv"]
    for k in ks:
        S.set_options(fixed_iters=k)
        N.set_options(fixed_iters=k)
        xs, info = S.solve(dev(b))
        xn, _ = N.solve(dev(b))
        assert info["status"] == ppcg.OK and info["iters"] == k, info
        assert np.array_equal(host(xs), host(xn)), (name, k)
        e = relerr(host(xs), oracle.pipecg(A, b, fixed_iters=k).x)
        print(f"{name} form {form} k={k}: {e:.2e}")
        assert e <= 1e-10, (k, e)
    S.close()
    N.close()


@pytest.mark.parametrize("name,tol", [("poisson3d_40", 1e-10), ("stencil27_40", 1e-9)])
def test_tolerance_solve_on_shared_lists(name, tol):
    A = ITER_CASES[name][0]()
    b = rhs_from_solution(A, xstar_uniform(A.n, 2))
    S = Solver(A, tol=tol, spmv_format="sell", flags=SH | FUSED)
    x, info = S.solve(dev(b))
    ref = oracle.pipecg(A, b, tol=tol)
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - ref.iters) <= 2, (info["iters"], ref.iters)
    assert oracle.true_relres(A, b, host(x)) <= tol
    S.close()


def test_batch_with_shared_lists_equals_solo_bitwise():
    mats = [poisson3d(30), poisson2d(100), stencil27_lognormal(32, seed=1), random_spd(9000, seed=2),
            poisson125(40), shifted(poisson2d(70), 0.2)]
    flags = [SH | FUSED, NOSH | FUSED, SH | TWO, SH, SH | FUSED, SH | TWO]
    bs = [rhs_from_solution(A, xstar_uniform(A.n, 30 + i)) for i, A in enumerate(mats)]
    solo = []
    for A, f, b in zip(mats, flags, bs):
        S = Solver(A, fixed_iters=33, spmv_format="sell", flags=f)
        solo.append(host(S.solve(dev(b))[0]))
        S.close()
    solvers = [Solver(A, fixed_iters=33, spmv_format="sell", flags=f) for A, f in zip(mats, flags)]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for i, (A, b, x, info) in enumerate(zip(mats, bs, xs, infos)):
        assert info["iters"] == 33, (i, info)
        assert np.array_equal(host(x), solo[i]), A.name
        assert relerr(host(x), oracle.pipecg(A, b, fixed_iters=33).x) <= 1e-10, A.name
    for S in solvers:
        S.close()


@pytest.mark.parametrize("gen", [lambda: poisson3d(40), lambda: stencil27_lognormal(40, seed=3)])
def test_fp32_values_on_shared_lists_equal_per_entry_columns(gen):
    """PIPECG with FP32 values (FP64 vectors, reliable updates) reads the
    lists too: the same products in the same order, so the solve to 1e-10
    equals the per-entry-column solve bit for bit."""
    A = gen()
    b = rhs_from_solution(A, xstar_uniform(A.n, 3))
    res = []
    for f in (SH, NOSH):
        S = Solver(A, tol=1e-10, precision="mixed_values", spmv_format="sell", flags=f)
        assert (S.matrix_info()["col_index_bytes"] == 0) == (f == SH)
        x, info = S.solve(dev(b))
        assert info["status"] == ppcg.OK
        assert oracle.true_relres(A, b, host(x)) <= 1e-10
        res.append((host(x), info["iters"], info["outer_iters"]))
        S.close()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1:] == res[1][1:]


@pytest.mark.parametrize("name", ["poisson3d_40", "stencil27_40", "poisson2d_600_three_rows"])
def test_classic_pcg_on_shared_lists(name):
    """Algorithm 1's SpMV (s = A p with p formed per gathered entry) reads the
    lists too: iterates equal the per-entry columns' bit for bit and meet the
    1e-10 bar against the oracle's Algorithm 1."""
    A = ITER_CASES[name][0]()
    b = rhs_from_solution(A, xstar_uniform(A.n, 4))
    S = Solver(A, fixed_iters=1, spmv_format="sell", method="pcg", flags=SH)
    N = Solver(A, fixed_iters=1, spmv_format="sell", method="pcg", flags=NOSH)
    assert S.matrix_info()["col_index_bytes"] == 0
    for k in (5, 40):
        S.set_options(fixed_iters=k)
        N.set_options(fixed_iters=k)
        xs, info = S.solve(dev(b))
        xn, _ = N.solve(dev(b))
        assert info["iters"] == k, info
        assert np.array_equal(host(xs), host(xn)), (name, k)
        assert relerr(host(xs), oracle.pcg(A, b, fixed_iters=k).x) <= 1e-10, (name, k)
    S.close()
    N.close()


@pytest.mark.parametrize("prec", ["mixed", "mixed_values"])
def test_classic_pcg_fp32_modes_on_shared_lists(prec):
    """FP32 Algorithm 1 (FP32 values and vectors, FP64 reliable updates) and
    Algorithm 1 with FP32 values: solves to 1e-10 on the lists equal those on
    per-entry columns bit for bit."""
    A = stencil27_lognormal(40, seed=3)
    b = rhs_from_solution(A, xstar_uniform(A.n, 5))
    res = []
    for f in (SH, NOSH):
        S = Solver(A, tol=1e-10, precision=prec, method="pcg", spmv_format="sell", flags=f)
        x, info = S.solve(dev(b))
        assert info["status"] == ppcg.OK, info
        assert oracle.true_relres(A, b, host(x)) <= 1e-10
        res.append((host(x), info["iters"], info["outer_iters"]))
        S.close()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1:] == res[1][1:]
