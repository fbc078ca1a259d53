"""The single-launch PIPECG iteration (one launch per iteration of Algorithm
2: SpMV into registers, the previous dot products reduced by every
workgroup, the fused updates of Section V-B) against the FP64 oracle through
the C ABI.

The form is forced with PPCG_FLAG_ITER_FUSED.  Its rows see the same rounded
operations as the two-launch form (SpMV in stored column order, the same
update formulas); only the association of the dot products differs, so
fixed iterates are held to the 1e-10 bar against the oracle, tolerance
solves to the oracle's iteration count within 2 and a true residual at or
below tol.  Cases span several fused tiles (512 to 2,048 rows) with a ragged last tile, the
value table, 16- and 32-bit columns, sorted rows, and the paths that end a
solve (restart, stagnation, breakdown).
"""

import os

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Solver, solve_batch
from workloads import (poisson125, poisson2d, poisson3d, random_spd, rhs_from_solution, shifted,
                       stencil27_lognormal, xstar_uniform)

pytestmark = pytest.mark.gpu

FUSED = ppcg.FLAG_ITER_FUSED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(A, seed=1):
    return rhs_from_solution(A, xstar_uniform(A.n, seed))


CASES = {
    # (generator, fixed iteration counts, extra create options)
    "c1_poisson2d_64": (lambda: poisson2d(64), (1, 10, 50, 100), {}),
    "poisson2d_100_ragged": (lambda: poisson2d(100), (3, 40, 120), {}),      # 10,000 rows: 19 tiles + 272
    "poisson3d_40": (lambda: poisson3d(40), (25, 100), {}),
    "stencil27_20_col16": (lambda: stencil27_lognormal(20, seed=3), (10, 20), {"flags": ppcg.FLAG_SELL_COL16}),
    "stencil27_20_col32": (lambda: stencil27_lognormal(20, seed=3), (10, 20), {"flags": ppcg.FLAG_SELL_COL32}),
    "random_spd_30001_sorted": (lambda: random_spd(30001, seed=5), (5, 30), {}),
    "poisson125_12_vtab": (lambda: poisson125(12), (5, 15), {"flags": ppcg.FLAG_SELL_VALUE_TABLE}),
    "tile_and_68_rows": (lambda: shifted(poisson2d(46), 0.1), (1, 7, 30), {}),  # 2,116 rows: 4 tiles + 68
    # 360,000 rows: 3 rows per thread (1,536-row tiles), 234 tiles + 576 rows
    "poisson2d_600_three_rows": (lambda: poisson2d(600), (4, 45), {}),
    # 200,000 rows: 2 rows per thread (1,024-row tiles), 195 tiles + 320 rows
    "random_spd_200000_two_rows": (lambda: random_spd(200000, seed=7), (6,), {}),
    # 1,906,624 rows on 256 compute units: 5 rows per thread (2,560-row
    # tiles, the tile model's choice), 744 tiles + 1,984 rows
    "poisson3d_124_five_rows": (lambda: poisson3d(124), (3, 12), {}),
    # 4,000,000 rows: 16 rows per thread (8,192-row tiles), 488 tiles + 2,304 rows
    "poisson2d_2000_sixteen_rows": (lambda: poisson2d(2000), (2, 9), {}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fixed_iterates_match_oracle(name):
    gen, ks, extra = CASES[name]
    A = gen()
    b = problem(A)
    flags = extra.get("flags", 0) | FUSED
    S = Solver(A, fixed_iters=1, spmv_format="sell", flags=flags)
    mi = S.matrix_info()
    assert mi["iter_launches"] == 1
    if extra.get("flags", 0) & ppcg.FLAG_SELL_VALUE_TABLE:
        assert mi["value_bytes"] == 1
    for k in ks:
        S.set_options(fixed_iters=k)
        x, info = S.solve(dev(b))
        assert info["status"] == ppcg.OK and info["iters"] == k, info
        ref = oracle.pipecg(A, b, fixed_iters=k)
        e = relerr(host(x), ref.x)
        print(f"{name} k={k}: {e:.2e}")
        assert e <= 1e-10, (k, e)
    S.close()


@pytest.mark.parametrize("name,tol", [("c1_poisson2d_64", 1e-8), ("poisson3d_40", 1e-10),
                                      ("random_spd_30001_sorted", 1e-10), ("stencil27_20_col16", 1e-9)])
def test_tolerance_solve_matches_oracle(name, tol):
    A = CASES[name][0]()
    b = problem(A)
    S = Solver(A, tol=tol, spmv_format="sell", flags=FUSED | CASES[name][2].get("flags", 0))
    x, info = S.solve(dev(b))
    ref = oracle.pipecg(A, b, tol=tol)
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - ref.iters) <= 2, (info["iters"], ref.iters)
    assert oracle.true_relres(A, b, host(x)) <= tol
    assert abs(info["rel_resid_true"] - oracle.true_relres(A, b, host(x))) <= 1e-3 * tol
    # solves are deterministic
    x2, info2 = S.solve(dev(b))
    assert np.array_equal(host(x2), host(x)) and info2["iters"] == info["iters"]
    S.close()


def test_paper_protocol_absolute_stop():
    A = poisson3d(32)
    b = rhs_from_solution(A, np.full(A.n, 1.0 / np.sqrt(A.n)))
    S = Solver(A, tol=1e-5, stop="abs", spmv_format="sell", flags=FUSED)
    x, info = S.solve(dev(b))
    ref = oracle.pipecg(A, b, tol=1e-5, stop=oracle.STOP_ABS)
    assert info["status"] == ppcg.OK and abs(info["iters"] - ref.iters) <= 2
    assert info["precond_norm"] < 1e-5


def test_restart_then_stagnation_and_breakdown_readings():
    """The endings of a solve take the same path as the two-launch form:
    restarts from x while the true residual misses tol, then STAGNATED; a
    breakdown near the attainable accuracy restarts too."""
    A = stencil27_lognormal(20, seed=2)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    refs = [oracle.pipecg(A, b, tol=1e-18, maxit=5000, max_restarts=2, dots=d) for d in ("seq", "comp")]
    S = Solver(A, tol=1e-18, max_iter=5000, max_restarts=2, spmv_format="sell", flags=FUSED)
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.STAGNATED and info["restarts"] == 2
    rel = oracle.true_relres(A, b, host(x))
    assert rel <= max(10 * max(r.rel_true for r in refs), 1e-14)
    S.close()
    S = Solver(A, tol=1e-14, max_iter=5000, max_restarts=3, spmv_format="sell", flags=FUSED)
    x, info = S.solve(dev(b))
    assert info["status"] in (ppcg.OK, ppcg.STAGNATED)
    assert oracle.true_relres(A, b, host(x)) <= 1e-13
    S.close()


def test_breakdown_at_first_iteration_is_reported():
    from workloads import CSR

    # indefinite, 6,000 rows so that the solve does not take the
    # one-workgroup kernel: a 2x2 block [[1, 2], [2, 1]] repeated
    nb = 3000
    rp = np.arange(0, 4 * nb + 1, 2, dtype=np.int32)
    ci = np.empty(4 * nb, np.int32)
    for k in range(nb):
        ci[4 * k:4 * k + 4] = [2 * k, 2 * k + 1, 2 * k, 2 * k + 1]
    val = np.tile([1.0, 2.0, 2.0, 1.0], nb)
    A = CSR(2 * nb, rp, ci, val)
    b = np.tile([1.0, -1.0], nb)
    ref = oracle.pipecg(A, b)
    S = Solver(A, tol=1e-8, spmv_format="sell", flags=FUSED)
    x, info = S.solve(dev(b))
    assert ref.status == oracle.BREAKDOWN
    assert info["status"] == ppcg.BREAKDOWN and info["iters"] == ref.iters == 0


def test_batch_mixes_forms_and_equals_solo_bitwise():
    """Fused, two-launch and one-workgroup systems in one batch: each result
    bitwise equal to its solo solve."""
    mats = [poisson2d(100), poisson3d(30), stencil27_lognormal(18, seed=4), poisson2d(40), random_spd(9000, seed=2)]
    flags = [FUSED, FUSED, ppcg.FLAG_ITER_TWO_LAUNCH, 0, FUSED]
    bs = [problem(A, seed=30 + i) for i, A in enumerate(mats)]
    solo = []
    for A, b, f in zip(mats, bs, flags):
        x, info = Solver(A, tol=1e-10, spmv_format="sell", flags=f).solve(dev(b))
        solo.append((host(x), info))
    solvers = [Solver(A, tol=1e-10, spmv_format="sell", flags=f) for A, f in zip(mats, flags)]
    assert [s.matrix_info()["iter_launches"] for s in solvers] == [1, 1, 2, 2, 1]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for (xs_, is_), x, info, A, b in zip(solo, xs, infos, mats, bs):
        assert np.array_equal(host(x), xs_), A.name
        assert info["iters"] == is_["iters"] and info["status"] == ppcg.OK
        assert oracle.true_relres(A, b, host(x)) <= 1e-10
        assert abs(info["iters"] - oracle.pipecg(A, b, tol=1e-10).iters) <= 2


def test_batch_fixed_iterates_match_oracle():
    mats = [poisson2d(100), random_spd(9000, seed=2), stencil27_lognormal(17, seed=1)]
    bs = [problem(A, seed=50 + i) for i, A in enumerate(mats)]
    solvers = [Solver(A, fixed_iters=33, spmv_format="sell", flags=FUSED) for A in mats]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for A, b, x, info in zip(mats, bs, xs, infos):
        assert info["iters"] == 33
        assert relerr(host(x), oracle.pipecg(A, b, fixed_iters=33).x) <= 1e-10


def test_kernel_timing_reports_the_single_launch():
    A = poisson3d(48)
    storage = ppcg.FLAG_SELL_COL32 | ppcg.FLAG_SELL_FULL_VALUES  # the same in both forms
    S = Solver(A, spmv_format="sell", flags=FUSED | storage)
    tf, ts = S.time_kernels(dev(problem(A)), iters=10)
    assert tf > 0 and ts == 0.0
    mi = S.matrix_info()
    # n is neither written nor read (16 bytes per row fewer than two
    # launches), and with a constant diagonal m is not written (8 more)
    T = Solver(A, spmv_format="sell", flags=ppcg.FLAG_ITER_TWO_LAUNCH | storage)
    assert mi["diag_const"] == 1
    assert abs((T.matrix_info()["bytes_per_iter"] - mi["bytes_per_iter"]) - 24.0 * A.n) < 1.0


def test_autotuned_form_is_correct():
    """Whatever form the autotuner picks for a system above the one-workgroup
    size, its iterates meet the bar."""
    A = poisson3d(64)
    b = problem(A)
    S = Solver(A, fixed_iters=60)
    assert S.matrix_info()["iter_launches"] in (1, 2)
    x, info = S.solve(dev(b))
    assert relerr(host(x), oracle.pipecg(A, b, fixed_iters=60).x) <= 1e-10


def _golden_c2():
    vals, meta = {}, {}
    with open(os.path.join(GOLDEN, "c2_poisson3d_128.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "x500":
                vals[int(p[1])] = float(p[2])
            else:
                meta[p[0]] = float(p[1])
    return vals, meta


def test_c2_full_size_fused():
    """128^3 7-point Poisson in the storage bench.py times: 500 fixed
    iterates (sampled against the oracle's golden values, and the norm) and
    the solve to 1e-10."""
    A = poisson3d(128)
    b = problem(A)
    vals, meta = _golden_c2()
    flags = FUSED | ppcg.FLAG_SELL_COL32 | ppcg.FLAG_SELL_FULL_VALUES
    S = Solver(A, fixed_iters=500, spmv_format="sell", flags=flags)
    x, info = S.solve(dev(b))
    assert info["iters"] == 500
    xh = host(x)
    idx = np.array(sorted(vals))
    assert relerr(xh[idx], np.array([vals[i] for i in idx])) <= 1e-10
    assert abs(np.linalg.norm(xh) - meta["norm_x500"]) <= 1e-10 * meta["norm_x500"]
    S.set_options(tol=1e-10)
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK and abs(info["iters"] - int(meta["tol1e-10_iters"])) <= 2
    assert info["rel_resid_true"] <= 1e-10
    S.close()
