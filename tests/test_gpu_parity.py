"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances.  The fused updates and the SpMV (SELL format) perform the same
rounded operations in the same order as the oracle, so the SpMV is checked
bit for bit.  The dot products are reduced in a different (fixed, tree)
order, so the scalars alpha and beta differ in their last bits and iterates
drift apart by rounding; for the well-conditioned cases here that drift stays
below 1e-10 relative after the fixed iteration counts tested, the bound set
for the FP64 iterates.  Tolerance solves are checked on the true residual and
on the iteration count (equal to the oracle's within 2).
"""

import ctypes
import math
import os

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import PPCGError, Server, Solver, solve_batch
from workloads import (CSR, batch_c4, poisson2d, poisson3d, random_spd, rhs_from_solution, shifted,
                       stencil27_lognormal, xstar_paper, xstar_uniform)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(A, seed=1):
    xs = xstar_uniform(A.n, seed)
    return rhs_from_solution(A, xs), xs


CASES = {
    "c1_poisson2d_64": lambda: poisson2d(64),
    "poisson2d_37_ragged": lambda: poisson2d(37),
    "poisson3d_24": lambda: poisson3d(24),
    "random_spd_3001": lambda: random_spd(3001, seed=2),
    "stencil27_12": lambda: stencil27_lognormal(12, seed=3),
}


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("fmt", ["sell", "csr_vector", "auto"])
def test_spmv_matches_oracle(name, fmt):
    A = CASES[name]()
    S = Solver(A, spmv_format=fmt)
    x = xstar_uniform(A.n, 7)
    y = host(S.spmv(dev(x)))
    y_ora = oracle.spmv(A, x)
    if S.matrix_info()["format"] == ppcg.SPMV_SELL:
        assert np.array_equal(y, y_ora), "SELL SpMV must match the oracle bit for bit"
    else:
        rowabs = np.abs(A.to_scipy()) @ np.abs(x)
        assert np.all(np.abs(y - y_ora) <= 4 * np.finfo(float).eps * rowabs)


def test_spmv_sorted_sell_is_bitwise():
    """Random SPD rows vary in length, so SELL sorts rows in windows
    (sigma > 1); the permuted product must still match bit for bit."""
    A = random_spd(5000, seed=9)
    S = Solver(A, spmv_format="sell")
    mi = S.matrix_info()
    assert mi["sell_sigma"] > 1
    assert mi["nnz_stored"] < 1.10 * A.nnz
    x = xstar_uniform(A.n, 3)
    assert np.array_equal(host(S.spmv(dev(x))), oracle.spmv(A, x))


@pytest.mark.parametrize("flags,expect16", [(ppcg.FLAG_SELL_COL16, True), (ppcg.FLAG_SELL_COL32, False),
                                            (0, None)])
def test_storage_choices_keep_results_exact(flags, expect16):
    """16-bit column offsets are used when every offset fits (forced, refused,
    or timed against 32-bit columns) and the constant diagonal of a Poisson
    matrix is read as one value; neither changes a single bit of the SpMV,
    and iterates still match the oracle.  The 27-point rows (odd length 27)
    and the ragged random rows exercise the odd-tail entry of the paired
    16-bit layout."""
    P = poisson3d(40)
    R = random_spd(70000, seed=1)  # random columns: offsets up to 70000, no 16-bit form
    for A, fits, const in ((P, True, 1), (R, False, 0), (random_spd(5000, seed=9), True, 0),
                           (stencil27_lognormal(20, seed=3), True, 0)):
        S = Solver(A, spmv_format="sell", flags=flags)
        mi = S.matrix_info()
        if expect16 is None or not fits:
            # 0: the chunks' shared offset lists (stencils in natural order)
            assert mi["col_index_bytes"] in ((0, 2, 4) if fits else (4,)), A.name
        else:
            assert mi["col_index_bytes"] == (2 if expect16 else 4), A.name
        assert mi["diag_const"] == const, A.name
        x = xstar_uniform(A.n, 3)
        assert np.array_equal(host(S.spmv(dev(x))), oracle.spmv(A, x))
        b, _ = problem(A)
        S.set_options(fixed_iters=15, spmv_format="sell")
        xg, _ = S.solve(dev(b))
        assert relerr(host(xg), oracle.pipecg(A, b, fixed_iters=15).x) <= 1e-10


@pytest.mark.parametrize("col_flag", [ppcg.FLAG_SELL_COL16, ppcg.FLAG_SELL_COL32])
def test_value_table_is_exact(col_flag):
    """A constant-coefficient stencil stores three values (6, -1 and the
    padding's 0).  With the value table forced, the PIPECG SpMV reads one-byte
    indices into it; the SpMV output, the solve to 1e-10 and its iteration
    count are bitwise those of the 8-byte values, with either column layout,
    for host and for device CSR input (the scan then copies the values in
    chunks)."""
    import torch

    A = poisson3d(40)
    b, _ = problem(A)
    x = xstar_uniform(A.n, 3)
    dev_csr = (torch.as_tensor(A.rp).cuda(), torch.as_tensor(A.ci).cuda(), torch.as_tensor(A.val).cuda())
    res = {}
    for label, src, vflag in (("on", A, ppcg.FLAG_SELL_VALUE_TABLE), ("on_dev", dev_csr, ppcg.FLAG_SELL_VALUE_TABLE),
                              ("off", A, ppcg.FLAG_SELL_FULL_VALUES)):
        S = Solver(src, spmv_format="sell", flags=col_flag | vflag, tol=1e-10)
        mi = S.matrix_info()
        y = host(S.spmv(dev(x)))
        xs, info = S.solve(dev(b))
        res[label] = (y, host(xs), info["iters"], mi)
        S.close()
    for label in ("on", "on_dev"):
        assert res[label][3]["value_bytes"] == 1 and res[label][3]["distinct_values"] == 3, label
    assert res["off"][3]["value_bytes"] == 8 and res["off"][3]["distinct_values"] == 0
    assert res["on"][3]["bytes_spmv"] < res["off"][3]["bytes_spmv"]
    assert np.array_equal(res["off"][0], oracle.spmv(A, x))
    for label in ("on", "on_dev"):
        assert np.array_equal(res[label][0], res["off"][0]), label
        assert np.array_equal(res[label][1], res["off"][1]), label
        assert res[label][2] == res["off"][2], label


def _tridiag_values(n, k):
    """SPD tridiagonal matrix with k distinct off-diagonal values (and the
    diagonal 4): k + 2 distinct stored values with the SELL padding."""
    import scipy.sparse as sp

    off = -1.0 - (np.arange(n - 1) % k) * 2.0 ** -10
    M = sp.diags([off, np.full(n, 4.0), off], [-1, 0, 1], format="csr")
    M.sort_indices()
    return CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64), f"tri{k}")


@pytest.mark.parametrize("n", [6000, 1_200_000])
def test_value_table_holds_at_most_256_values(n):
    """254 off-diagonal values + 4 + the padding's 0 = 256 fit the one-byte
    table; one more value and the matrix keeps its 8-byte values.  Either way
    the SpMV equals the oracle's bit for bit.  At 1.2M rows (3.6M values) the
    scan runs on several host threads whose value sets are merged."""
    for k, fits in ((254, True), (255, False)):
        A = _tridiag_values(n, k)
        S = Solver(A, spmv_format="sell", flags=ppcg.FLAG_SELL_VALUE_TABLE)
        mi = S.matrix_info()
        assert mi["distinct_values"] == (256 if fits else 0), k
        assert mi["value_bytes"] == (1 if fits else 8), k
        x = xstar_uniform(A.n, 4)
        assert np.array_equal(host(S.spmv(dev(x))), oracle.spmv(A, x)), k
        S.close()


# ---------------------------------------------------------------- fixed iterates

@pytest.mark.parametrize("name,ks", [("c1_poisson2d_64", (1, 10, 50, 100)), ("poisson2d_37_ragged", (5, 40)),
                                     ("poisson3d_24", (20, 60)), ("random_spd_3001", (10, 30)),
                                     ("stencil27_12", (10, 20))])
@pytest.mark.parametrize("fmt", ["sell", "csr_vector"])
def test_fixed_iterates_match_oracle(name, ks, fmt):
    A = CASES[name]()
    b, _ = problem(A)
    S = Solver(A, spmv_format=fmt)
    bd = dev(b)
    for k in ks:
        S.set_options(fixed_iters=k)
        x, info = S.solve(bd)
        ref = oracle.pipecg(A, b, fixed_iters=k)
        assert info["status"] == ppcg.OK
        assert info["iters"] == k == ref.iters
        assert relerr(host(x), ref.x) <= 1e-10, (k, relerr(host(x), ref.x))


def test_solves_are_deterministic():
    A = random_spd(4000, seed=4)
    b, _ = problem(A)
    S = Solver(A, fixed_iters=40)
    x1, _ = S.solve(dev(b))
    x2, _ = S.solve(dev(b))
    assert np.array_equal(host(x1), host(x2))


# ---------------------------------------------------------------- tolerance solves

@pytest.mark.parametrize("name,tol", [("c1_poisson2d_64", 1e-8), ("poisson3d_24", 1e-10),
                                      ("random_spd_3001", 1e-10), ("stencil27_12", 1e-8)])
def test_tolerance_solve_matches_oracle(name, tol):
    A = CASES[name]()
    b, xs = problem(A)
    S = Solver(A, tol=tol)
    x, info = S.solve(dev(b))
    ref = oracle.pipecg(A, b, tol=tol)
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - ref.iters) <= 2
    assert info["rel_resid_true"] <= tol
    assert oracle.true_relres(A, b, host(x)) <= tol


def test_paper_protocol_absolute_preconditioned_tolerance():
    """Section VI protocol: x* = 1/sqrt(N), b = A x*, absolute tolerance 1e-5
    on sqrt((u,u)), at most 10000 iterations."""
    for A in (poisson2d(64), poisson3d(32)):
        b = rhs_from_solution(A, xstar_paper(A.n))
        S = Solver(A, tol=1e-5, stop="abs", max_iter=10000)
        x, info = S.solve(dev(b))
        ref = oracle.pipecg(A, b, tol=1e-5, stop=oracle.STOP_ABS, maxit=10000)
        assert info["status"] == ppcg.OK
        assert abs(info["iters"] - ref.iters) <= 2
        assert info["precond_norm"] < 1e-5


# ---------------------------------------------------------------- full size 128^3

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


@pytest.fixture(scope="module")
def c2():
    A = poisson3d(128)
    b, _ = problem(A)
    return A, b


# the storage and iteration form bench.py pins for this matrix (16-bit
# columns, one-byte value table, one launch per iteration), 32-bit columns
# with 8-byte values in both iteration forms, the chunks' shared offset lists
# with the value table, and the autotuner's own choice
C2_STORAGE = {"bench": dict(spmv_format="sell", flags=ppcg.FLAG_SELL_COL16 | ppcg.FLAG_SELL_VALUE_TABLE |
                            ppcg.FLAG_ITER_FUSED),
              "full_values_fused": dict(spmv_format="sell", flags=ppcg.FLAG_SELL_COL32 | ppcg.FLAG_SELL_FULL_VALUES |
                                        ppcg.FLAG_ITER_FUSED),
              "two_launch": dict(spmv_format="sell", flags=ppcg.FLAG_SELL_COL32 | ppcg.FLAG_SELL_FULL_VALUES |
                                 ppcg.FLAG_ITER_TWO_LAUNCH),
              "shared_offsets_fused": dict(spmv_format="sell", flags=ppcg.FLAG_SELL_SHARED_OFFSETS |
                                           ppcg.FLAG_SELL_VALUE_TABLE | ppcg.FLAG_ITER_FUSED),
              "auto": {}}


@pytest.mark.parametrize("storage", sorted(C2_STORAGE))
def test_c2_full_size_spmv_bitwise(c2, storage):
    A, _ = c2
    S = Solver(A, **C2_STORAGE[storage])
    x = xstar_uniform(A.n, 5)
    assert np.array_equal(host(S.spmv(dev(x))), oracle.spmv(A, x))


@pytest.mark.parametrize("storage", sorted(C2_STORAGE))
def test_c2_full_size_500_iterations_sampled(c2, storage):
    A, b = c2
    vals, meta = _golden_c2()
    S = Solver(A, fixed_iters=500, **C2_STORAGE[storage])
    x, info = S.solve(dev(b))
    assert info["iters"] == 500
    xh = host(x)
    idx = np.array(sorted(vals))
    ref = np.array([vals[i] for i in idx])
    assert relerr(xh[idx], ref) <= 1e-10
    assert abs(np.linalg.norm(xh) - meta["norm_x500"]) <= 1e-10 * meta["norm_x500"]


@pytest.mark.parametrize("storage", sorted(C2_STORAGE))
def test_c2_full_size_to_tolerance(c2, storage):
    A, b = c2
    _, meta = _golden_c2()
    S = Solver(A, tol=1e-10, **C2_STORAGE[storage])
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - int(meta["tol1e-10_iters"])) <= 2
    assert info["rel_resid_true"] <= 1e-10


# ---------------------------------------------------------------- edge cases

def test_one_by_one_and_tiny_systems():
    A = CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    x, info = Solver(A).solve(dev([2.0]))
    assert info["iters"] == 1 and host(x)[0] == 0.5
    D = np.array([[4.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 4.0]])
    from scipy.sparse import csr_matrix

    M = csr_matrix(D)
    A3 = CSR(3, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)
    b = np.array([1.0, 2.0, 3.0])
    x, info = Solver(A3, tol=1e-14).solve(dev(b))
    assert info["iters"] <= 3
    assert relerr(host(x), np.linalg.solve(D, b)) <= 1e-14


def test_maxit_zero_zero_rhs_and_converged_guess():
    A = poisson2d(20)
    b, xs = problem(A)
    x, info = Solver(A, max_iter=0).solve(dev(b))
    assert info["status"] == ppcg.NOT_CONVERGED and info["iters"] == 0 and np.all(host(x) == 0)
    x, info = Solver(A).solve(dev(np.zeros(A.n)))
    assert info["status"] == ppcg.OK and info["iters"] == 0 and np.all(host(x) == 0)
    bx = oracle.spmv(A, xs)
    x, info = Solver(A, tol=1e-12).solve(dev(bx), x0=dev(xs))
    assert info["iters"] == 0 and np.array_equal(host(x), xs)


def test_tol_zero_runs_to_maxit():
    A = poisson2d(16)
    b, _ = problem(A)
    x, info = Solver(A, tol=0.0, max_iter=25).solve(dev(b))
    ref = oracle.pipecg(A, b, tol=0.0, maxit=25)
    assert info["status"] == ref.status
    assert info["iters"] == ref.iters


def test_x0_aliases_x_and_nonzero_initial_guess():
    A = random_spd(2000, seed=5)
    b, _ = problem(A)
    g = xstar_uniform(A.n, 11) * 0.5
    S = Solver(A, fixed_iters=15)
    xt = dev(g)
    x, _ = S.solve(dev(b), x0=xt, out=xt)
    ref = oracle.pipecg(A, b, x0=g, fixed_iters=15)
    assert relerr(host(x), ref.x) <= 1e-10


def test_host_vectors_and_device_csr():
    import torch

    A = poisson2d(30)
    b, _ = problem(A)
    S = Solver(A, fixed_iters=20, vec_mem="host")
    xh = torch.zeros(A.n, dtype=torch.float64)
    S.solve(torch.as_tensor(b), out=xh)
    ref = oracle.pipecg(A, b, fixed_iters=20)
    assert relerr(xh.numpy(), ref.x) <= 1e-10
    Ad = (dev(A.rp).to(torch.int32), dev(A.ci).to(torch.int32), dev(A.val))
    S2 = Solver(Ad, fixed_iters=20)
    x2, _ = S2.solve(dev(b))
    assert np.array_equal(host(x2), xh.numpy())


def _bad(A, **edit):
    rp, ci, val = A.rp.copy(), A.ci.copy(), A.val.copy()
    if "rp" in edit:
        rp = edit["rp"](rp)
    if "ci" in edit:
        ci = edit["ci"](ci)
    if "val" in edit:
        val = edit["val"](val)
    return CSR(A.n, rp, ci, val)


@pytest.mark.parametrize("what", ["diag_missing", "diag_negative", "col_range", "col_order", "rp0", "nan"])
def test_bad_csr_rejected(what):
    A = poisson2d(6)
    if what == "diag_missing":
        # replace row 0's diagonal column by a duplicate-free off-diagonal slot
        B = _bad(A, ci=lambda c: np.where(np.arange(c.size) == 0, 2, c))
    elif what == "diag_negative":
        B = _bad(A, val=lambda v: np.where(v == 4.0, -4.0, v))
    elif what == "col_range":
        B = _bad(A, ci=lambda c: np.where(np.arange(c.size) == 5, A.n + 3, c))
    elif what == "col_order":
        B = _bad(A, ci=lambda c: np.concatenate([[c[1], c[0]], c[2:]]))
    elif what == "rp0":
        B = _bad(A, rp=lambda r: np.concatenate([[1], r[1:]]).astype(np.int32))
    else:
        B = _bad(A, val=lambda v: np.where(np.arange(v.size) == 7, np.nan, v))
    with pytest.raises(PPCGError) as e:
        Solver(B)
    assert e.value.status == ppcg.ERR_BAD_CSR


def test_indefinite_matrix_breaks_down():
    D = np.array([[1.0, 2.0], [2.0, 1.0]])
    A = CSR(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), D.ravel())
    x, info = Solver(A).solve(dev([1.0, -1.0]))
    assert info["status"] == ppcg.BREAKDOWN


def test_kernel_timing_entry_point():
    A = poisson3d(48)
    b, _ = problem(A)
    for flags in (ppcg.FLAG_ITER_TWO_LAUNCH, 0):
        S = Solver(A, flags=flags)
        tv, ts = S.time_kernels(dev(b), iters=10)
        # the single-launch form reports its one kernel in the first figure
        assert tv > 0 and (ts > 0 if S.matrix_info()["iter_launches"] == 2 else ts == 0.0)


# ---------------------------------------------------------------- batching

def _batch_systems():
    mats = [shifted(poisson2d(s), h) for s, h in [(33, 0.01), (64, 0.2), (17, 0.0), (90, 0.05)]]
    mats += [random_spd(3001, seed=8), poisson3d(21)]
    return mats


def test_batch_results_bitwise_equal_solo():
    mats = _batch_systems()
    bs = [problem(A, seed=20 + i)[0] for i, A in enumerate(mats)]
    solo = []
    for A, b in zip(mats, bs):
        x, info = Solver(A, tol=1e-10).solve(dev(b))
        solo.append((host(x), info))
    solvers = [Solver(A, tol=1e-10) for A in mats]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for (xs_, is_), x, info, A, b in zip(solo, xs, infos, mats, bs):
        assert np.array_equal(host(x), xs_), A.name
        assert info["iters"] == is_["iters"]
        assert info["status"] == ppcg.OK
        assert info["rel_resid_true"] <= 1e-10
        ref = oracle.pipecg(A, b, tol=1e-10)
        assert abs(info["iters"] - ref.iters) <= 2


def test_batch_c4_subset_against_oracle():
    spec = [s for s in batch_c4(seed=0)][:12]
    mats = [shifted(poisson2d(min(side, 96)), sh) for side, sh in spec]
    bs = [problem(A, seed=100 + i)[0] for i, A in enumerate(mats)]
    solvers = [Solver(A, tol=1e-10) for A in mats]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for A, b, x, info in zip(mats, bs, xs, infos):
        assert info["status"] == ppcg.OK
        assert oracle.true_relres(A, b, host(x)) <= 1e-10
        ref = oracle.pipecg(A, b, tol=1e-10)
        assert abs(info["iters"] - ref.iters) <= 2


def test_batch_fixed_iterates_match_oracle():
    mats = _batch_systems()
    bs = [problem(A, seed=40 + i)[0] for i, A in enumerate(mats)]
    solvers = [Solver(A, fixed_iters=25) for A in mats]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for A, b, x in zip(mats, bs, xs):
        assert relerr(host(x), oracle.pipecg(A, b, fixed_iters=25).x) <= 1e-10


# ---------------------------------------------------------------- mixed precision

@pytest.mark.parametrize("gen", [lambda: stencil27_lognormal(16, seed=1), lambda: poisson2d(64),
                                 lambda: random_spd(20000, seed=3)])
def test_mixed_precision_reaches_fp64_tolerance(gen):
    """FP32 vectors and values with the default method: the library iterates
    with Algorithm 1 (reported in the info) and reaches the FP64 tolerance."""
    A = gen()
    b, xs = problem(A)
    S = Solver(A, tol=1e-10, precision="mixed")
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK, info
    assert info["method"] == ppcg.METHOD_PCG and info["precision"] == ppcg.MIXED_FP32
    assert info["outer_iters"] >= 1
    assert info["rel_resid_true"] <= 1e-10
    assert oracle.true_relres(A, b, host(x)) <= 1e-10
    ref = oracle.pipecg(A, b, tol=1e-10)
    # both solutions satisfy the same residual bound; their distance is bounded
    # by the conditioning times the tolerance
    assert relerr(host(x), ref.x) <= 1e-5


# ---------------------------------------------------------------- serving

def _serve_all(srv, reqs, stagger=2):
    """Submit requests a few at a time between steps; return id -> result."""
    ids = {}
    pending = list(reqs)
    results = {}
    while pending or len(results) < len(ids):
        for _ in range(stagger):
            if pending:
                key, A, b, tol, prec = pending.pop(0)
                ids[srv.submit(A, b, tol, prec)] = key
        srv.step()
        for rid, key in list(ids.items()):
            if key in results:
                continue
            r = srv.poll(rid)
            if r is not None:
                results[key] = r
    return results


def test_server_result_same_alone_and_in_mix():
    A = poisson3d(20)
    b, _ = problem(A, 3)
    alone = _serve_all(Server(), [("R", A, b, 1e-10, "fp64")])["R"]
    mix = [("m0", random_spd(4000, seed=1), problem(random_spd(4000, seed=1))[0], 1e-8, "fp64"),
           ("R", A, b, 1e-10, "fp64"),
           ("m1", poisson2d(50), problem(poisson2d(50))[0], 1e-6, "fp64"),
           ("m2", stencil27_lognormal(10, seed=2), problem(stencil27_lognormal(10, seed=2))[0], 1e-10, "mixed"),
           ("m4", stencil27_lognormal(11, seed=5), problem(stencil27_lognormal(11, seed=5))[0], 1e-10,
            "mixed_values"),
           ("m3", poisson2d(120), problem(poisson2d(120))[0], 1e-10, "fp64")]
    res = _serve_all(Server(), mix, stagger=1)
    assert np.array_equal(res["R"][0], alone[0])
    assert res["R"][1]["iters"] == alone[1]["iters"]
    for key, Am, bm, tol, prec in mix:
        assert res[key][1]["status"] == ppcg.OK
        assert oracle.true_relres(Am, bm, res[key][0]) <= tol
    # the served result equals a direct solve of the same request
    x, info = Solver(A, tol=1e-10).solve(dev(b))
    assert np.array_equal(host(x), alone[0])


def test_server_refuses_over_budget_and_admits_in_turn():
    A = poisson2d(100)
    b, _ = problem(A)
    fp = ppcg.footprint_bytes(A.n, A.nnz)
    srv = Server(budget_bytes=1.5 * fp)
    big = poisson2d(200)
    with pytest.raises(PPCGError) as e:
        srv.submit(big, problem(big)[0], 1e-8)
    assert e.value.status == ppcg.ERR_BUDGET
    # all four queued at once; the budget holds one at a time, also while a
    # finished one is still being copied out and released (counted as active)
    ids = [srv.submit(A, b, 1e-8) for _ in range(4)]
    xs, most = {}, 0
    while len(xs) < 4:
        active, queued = srv.step()
        most = max(most, active)
        for rid in ids:
            if rid not in xs:
                r = srv.poll(rid)
                if r is not None:
                    xs[rid] = r[0]
    assert most == 1
    xs = list(xs.values())
    for x in xs[1:]:
        assert np.array_equal(x, xs[0])


def test_server_bad_request_fails_alone():
    """A request whose matrix fails validation (a negative diagonal entry)
    ends with ERR_BAD_CSR on its own; the requests before and after it are
    prepared, solved and returned as if it were not there."""
    good = poisson2d(40)
    bad = CSR(good.n, good.rp, good.ci, good.val.copy(), "bad")
    d = [k for i in range(bad.n) for k in range(bad.rp[i], bad.rp[i + 1]) if bad.ci[k] == i]
    bad.val[d[7]] = -1.0
    b = problem(good)[0]
    alone = _serve_all(Server(), [("g", good, b, 1e-10, "fp64")])["g"]
    srv = Server()
    ids = [srv.submit(good, b, 1e-10), srv.submit(bad, b, 1e-10), srv.submit(good, b, 1e-10)]
    done = {}
    while len(done) < 3:
        srv.step()
        for rid in ids:
            if rid in done:
                continue
            try:
                r = srv.poll(rid)
            except PPCGError as e:
                r = e.status
            if r is not None:
                done[rid] = r
    assert done[ids[1]] == ppcg.ERR_BAD_CSR
    for rid in (ids[0], ids[2]):
        assert done[rid][1]["status"] == ppcg.OK
        assert np.array_equal(done[rid][0], alone[0])
    srv.close()


def test_server_many_requests_match_direct_solves():
    """48 requests of mixed kinds and sizes (small-system kernel, batched
    tiles, several tolerances) arrive in bursts between steps, so that
    preparation, admission, retirement and the copy-out interleave: every
    served solution equals a direct solve of the same request bit for bit."""
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(48):
        k = i % 3
        if k == 0:
            A = poisson2d(int(rng.integers(8, 80)))
        elif k == 1:
            A = poisson3d(int(rng.integers(5, 24)))
        else:
            A = random_spd(int(rng.integers(300, 20000)), seed=int(rng.integers(1 << 20)))
        tol = float(rng.choice([1e-6, 1e-8, 1e-10]))
        reqs.append((f"q{i}", A, problem(A, 100 + i)[0], tol, "fp64"))
    res = _serve_all(Server(), reqs, stagger=5)
    assert len(res) == len(reqs)
    for key, A, b, tol, _ in reqs:
        xs, info = res[key]
        assert info["status"] == ppcg.OK, (key, info)
        S = Solver(A, tol=tol)
        xd, infod = S.solve(dev(b))
        S.close()
        assert np.array_equal(xs, host(xd)), key
        assert info["iters"] == infod["iters"], key


def test_server_borrowing_inputs_gives_the_same_results():
    """A server created with PPCG_FLAG_BORROW_INPUTS reads the caller's
    arrays instead of copies: same results, bit for bit."""
    mats = [poisson3d(16), random_spd(3000, seed=4), poisson2d(45)]
    reqs = [(f"r{i}", A, problem(A, 30 + i)[0], 1e-10, "fp64") for i, A in enumerate(mats)]
    copied = _serve_all(Server(), reqs)
    borrowed = _serve_all(Server(borrow=True), reqs)
    for key, *_ in reqs:
        assert np.array_equal(copied[key][0], borrowed[key][0])
        assert copied[key][1]["iters"] == borrowed[key][1]["iters"]


def test_server_automatic_precision():
    """Automatic precision: a large request runs with FP32 values (it makes
    reliable updates), a small one in FP64; both reach the tolerance."""
    big, small = stencil27_lognormal(41, seed=1), poisson2d(40)
    reqs = [("big", big, problem(big)[0], 1e-10, "auto"), ("small", small, problem(small)[0], 1e-10, "auto")]
    res = _serve_all(Server(), reqs)
    for key, A, b, tol, _ in reqs:
        assert res[key][1]["status"] == ppcg.OK
        assert oracle.true_relres(A, b, res[key][0]) <= tol
    assert res["big"][1]["outer_iters"] >= 1
    assert res["small"][1]["outer_iters"] == 0
    assert res["big"][1]["precision"] == ppcg.MIXED_FP32_VALUES
    assert res["small"][1]["precision"] == ppcg.FP64
    assert res["big"][1]["method"] == res["small"][1]["method"] == ppcg.METHOD_PIPECG


def test_server_automatic_precision_takes_fp32_pcg_for_large_systems():
    """At 262144 rows and more the server runs classic PCG in FP32 (values and
    vectors) with FP64 reliable updates; it reaches the FP64 tolerance."""
    big = poisson3d(64)
    b = problem(big)[0]
    x, info = _serve_all(Server(), [("big", big, b, 1e-10, "auto")])["big"]
    assert info["status"] == ppcg.OK, info
    assert info["precision"] == ppcg.MIXED_FP32 and info["method"] == ppcg.METHOD_PCG
    assert info["outer_iters"] >= 2
    assert oracle.true_relres(big, b, x) <= 1e-10


def test_server_automatic_precision_falls_back_to_fp64():
    """With reliable updates switched off (no pause, no update allowed), the
    FP32-values run of a matrix whose values FP32 does not represent ends
    above tol (STAGNATED); the server reruns it in FP64 from its last
    iterate, which then needs fewer iterations than a solve from zero."""
    big = stencil27_lognormal(48, seed=1)
    b = problem(big)[0]
    res = _serve_all(Server(inner_tol=1e-30, max_outer=0), [("big", big, b, 1e-10, "auto")])
    x, info = res["big"]
    assert info["status"] == ppcg.OK
    assert oracle.true_relres(big, b, x) <= 1e-10
    assert info["outer_iters"] == 0
    assert info["precision"] == ppcg.FP64 and info["method"] == ppcg.METHOD_PIPECG
    assert info["iters"] < 0.8 * oracle.pipecg(big, b, tol=1e-10).iters


def test_server_automatic_fp32_pcg_falls_back_to_fp64_when_budget_spent():
    """One reliable-update stretch allowed (max_outer 1, pause at 0.1): the
    FP32 classic-PCG run ends NOT_CONVERGED with its refinement budget spent,
    and the server reruns the request in FP64 PIPECG from its last iterate."""
    big = poisson3d(64)
    b = problem(big)[0]
    x, info = _serve_all(Server(inner_tol=0.1, max_outer=1), [("big", big, b, 1e-10, "auto")])["big"]
    assert info["status"] == ppcg.OK, info
    assert info["precision"] == ppcg.FP64 and info["method"] == ppcg.METHOD_PIPECG
    assert oracle.true_relres(big, b, x) <= 1e-10
    assert info["iters"] < oracle.pipecg(big, b, tol=1e-10).iters


# ---------------------------------------------------------------- FP32 values + reliable updates

def _round32(A):
    return CSR(A.n, A.rp, A.ci, A.val.astype(np.float32).astype(np.float64), A.name + "_fp32")


def _diag_fp32_exact(A):
    """A with its diagonal rounded to FP32 (still SPD: the change is ~1e-7
    relative, far below the diagonal-dominance margin)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    val = A.val.copy()
    on = A.ci == rows
    val[on] = val[on].astype(np.float32).astype(np.float64)
    return CSR(A.n, A.rp, A.ci, val, A.name)


@pytest.mark.parametrize("gen", [lambda: stencil27_lognormal(14, seed=2), lambda: random_spd(5000, seed=6)])
def test_fp32_values_iterates_match_oracle_on_rounded_matrix(gen):
    """Before the first reliable update the iteration is PIPECG on the
    FP32-rounded operator (FP64 vectors, FP64 accumulation); with x0 = 0 the
    initial residual is b either way, so the oracle run on the rounded matrix
    is the reference.  The diagonal is made FP32-exact so that both sides use
    the same Jacobi preconditioner.  The GPU evaluates alpha's denominator
    directly instead of by the recurrence (equal in exact arithmetic), so the
    iterates agree to rounding."""
    A = _diag_fp32_exact(gen())
    b, _ = problem(A)
    S = Solver(A, precision="mixed_values", inner_tol=1e-30, spmv_format="sell")
    for k in (1, 4, 12):
        S.set_options(precision="mixed_values", fixed_iters=k, inner_tol=1e-30)
        x, info = S.solve(dev(b))
        ref = oracle.pipecg(_round32(A), b, fixed_iters=k)
        assert info["iters"] == k and info["outer_iters"] == 0
        assert relerr(host(x), ref.x) <= 1e-10, k


@pytest.mark.parametrize("gen,factor", [(lambda: stencil27_lognormal(16, seed=1), 1e-3),
                                        (lambda: stencil27_lognormal(16, seed=1), 0.3),
                                        (lambda: poisson3d(24), 1e-2),
                                        (lambda: random_spd(20000, seed=3), 1e-3)])
def test_fp32_values_reliable_updates_reach_fp64_tolerance(gen, factor):
    A = gen()
    b, _ = problem(A)
    S = Solver(A, tol=1e-10, precision="mixed_values", inner_tol=factor)
    x, info = S.solve(dev(b))
    ref = oracle.pipecg(A, b, tol=1e-10)
    assert info["status"] == ppcg.OK, info
    assert info["rel_resid_true"] <= 1e-10
    assert oracle.true_relres(A, b, host(x)) <= 1e-10
    # one Krylov sequence: the iteration count stays close to the FP64 one
    assert info["iters"] <= 1.15 * ref.iters + 5, (info["iters"], ref.iters)
    assert relerr(host(x), ref.x) <= 1e-5


def test_fp32_values_batch_bitwise_equals_solo():
    mats = [stencil27_lognormal(12, seed=4), shifted(poisson2d(70), 0.01), random_spd(4000, seed=2)]
    bs = [problem(A, seed=60 + i)[0] for i, A in enumerate(mats)]
    solo = [host(Solver(A, tol=1e-10, precision="mixed_values").solve(dev(b))[0]) for A, b in zip(mats, bs)]
    solvers = [Solver(A, tol=1e-10, precision="mixed_values") for A in mats]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for x, xs_, info in zip(xs, solo, infos):
        assert np.array_equal(host(x), xs_)
        assert info["status"] == ppcg.OK and info["rel_resid_true"] <= 1e-10


@pytest.mark.parametrize("gen", [lambda: poisson2d(64), lambda: poisson2d(37), lambda: shifted(poisson3d(14), 0.1)])
def test_small_kernel_matrix_in_lds_is_bitwise(gen):
    """The one-workgroup kernel stages a matrix with a value table in LDS
    (16-bit column offsets and one-byte value indices) and reads nothing else
    per iteration; with 8-byte values forced it reads the matrix from memory.
    Both add the same products in the same order: the solves are equal bit
    for bit, and meet the tolerance."""
    A = gen()
    b, _ = problem(A)
    res = []
    for vflag in (ppcg.FLAG_SELL_VALUE_TABLE, ppcg.FLAG_SELL_FULL_VALUES):
        S = Solver(A, tol=1e-10, spmv_format="sell", flags=vflag)
        assert S.matrix_info()["value_bytes"] == (1 if vflag == ppcg.FLAG_SELL_VALUE_TABLE else 8)
        x, info = S.solve(dev(b))
        assert info["status"] == ppcg.OK
        assert oracle.true_relres(A, b, host(x)) <= 1e-10
        res.append((host(x), info["iters"]))
        S.close()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]
