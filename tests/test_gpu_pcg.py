"""GPU parity of the classic PCG path (Algorithm 1, method="pcg") against the
oracle's Algorithm 1, through the C ABI.

The SpMV forms the direction p = u + beta p for every gathered entry with the
same rounded operations as the oracle, and rows are summed in CSR order
(SELL), so differences come only from the order of the dot-product
reductions, as for the pipelined path: FP64 iterates are held to 1e-10
relative after fixed iteration counts, tolerance solves to the oracle's
iteration count within 2.
"""

import os

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import PPCGError, Solver, solve_batch
from workloads import (CSR, poisson2d, poisson3d, random_spd, rhs_from_solution, shifted, stencil27_lognormal,
                       xstar_paper, xstar_uniform)

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
    return rhs_from_solution(A, xstar_uniform(A.n, seed))


CASES = {
    "c1_poisson2d_64": lambda: poisson2d(64),
    "poisson2d_37_ragged": lambda: poisson2d(37),
    "poisson3d_24": lambda: poisson3d(24),
    "random_spd_3001": lambda: random_spd(3001, seed=2),
    "stencil27_12": lambda: stencil27_lognormal(12, seed=3),
}


@pytest.mark.parametrize("name,ks", [("c1_poisson2d_64", (1, 2, 3, 10, 51)), ("poisson2d_37_ragged", (5, 40)),
                                     ("poisson3d_24", (20, 61)), ("random_spd_3001", (10, 30)),
                                     ("stencil27_12", (7, 20))])
@pytest.mark.parametrize("fmt", ["sell", "csr_vector"])
def test_pcg_fixed_iterates_match_oracle(name, ks, fmt):
    """Odd and even counts: the direction alternates between two buffers."""
    A = CASES[name]()
    b = problem(A)
    S = Solver(A, spmv_format=fmt, method="pcg")
    for k in ks:
        S.set_options(fixed_iters=k, method="pcg")
        x, info = S.solve(dev(b))
        ref = oracle.pcg(A, b, fixed_iters=k)
        assert info["status"] == ppcg.OK
        assert info["iters"] == k == ref.iters
        assert relerr(host(x), ref.x) <= 1e-10, (k, relerr(host(x), ref.x))


@pytest.mark.parametrize("name,tol", [("c1_poisson2d_64", 1e-8), ("poisson3d_24", 1e-10),
                                      ("random_spd_3001", 1e-10), ("stencil27_12", 1e-8)])
def test_pcg_tolerance_solve_matches_oracle(name, tol):
    A = CASES[name]()
    b = problem(A)
    x, info = Solver(A, tol=tol, method="pcg").solve(dev(b))
    ref = oracle.pcg(A, b, tol=tol)
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - ref.iters) <= 2
    assert info["rel_resid_true"] <= tol
    assert oracle.true_relres(A, b, host(x)) <= tol


def test_pcg_paper_protocol_absolute_tolerance():
    A = poisson3d(32)
    b = rhs_from_solution(A, xstar_paper(A.n))
    x, info = Solver(A, tol=1e-5, stop="abs", max_iter=10000, method="pcg").solve(dev(b))
    ref = oracle.pcg(A, b, tol=1e-5, stop=oracle.STOP_ABS, maxit=10000)
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - ref.iters) <= 2
    assert info["precond_norm"] < 1e-5


def test_pcg_and_pipecg_agree_at_tolerance():
    """Algorithms 1 and 2 are the same method in exact arithmetic."""
    A = stencil27_lognormal(16, seed=5)
    b = problem(A)
    x1, i1 = Solver(A, tol=1e-10, method="pcg").solve(dev(b))
    x2, i2 = Solver(A, tol=1e-10).solve(dev(b))
    assert abs(i1["iters"] - i2["iters"]) <= 3
    assert relerr(host(x1), host(x2)) <= 1e-6


def _golden(name):
    vals, meta = {}, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "x500":
                vals[int(p[1])] = float(p[2])
            else:
                meta[p[0]] = float(p[1])
    return vals, meta


def test_pcg_c2_full_size():
    """3-D 7-point Poisson 128^3: 500 iterations on sampled entries, and the
    solve to 1e-10, against values the oracle's Algorithm 1 wrote."""
    A = poisson3d(128)
    b = problem(A)
    vals, meta = _golden("c2_poisson3d_128_pcg.txt")
    S = Solver(A, fixed_iters=500, method="pcg")
    x, info = S.solve(dev(b))
    assert info["iters"] == 500
    xh = host(x)
    idx = np.array(sorted(vals))
    assert relerr(xh[idx], np.array([vals[i] for i in idx])) <= 1e-10
    assert abs(np.linalg.norm(xh) - meta["norm_x500"]) <= 1e-10 * meta["norm_x500"]
    S.set_options(tol=1e-10, method="pcg")
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - int(meta["tol1e-10_iters"])) <= 2
    assert info["rel_resid_true"] <= 1e-10


def test_pcg_edge_cases():
    A = CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    x, info = Solver(A, method="pcg").solve(dev([2.0]))
    assert info["iters"] == 1 and host(x)[0] == 0.5
    A = poisson2d(16)
    S = Solver(A, method="pcg")
    x, info = S.solve(dev(np.zeros(A.n)))  # zero right-hand side: x = 0 at once
    assert info["iters"] == 0 and not np.any(host(x))
    b = problem(A)
    S.set_options(max_iter=0, method="pcg")
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.NOT_CONVERGED and info["iters"] == 0
    # an indefinite matrix breaks down at once: (p, A p) <= 0
    D = CSR(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([1.0, 3.0, 3.0, 1.0]))
    x, info = Solver(D, method="pcg").solve(dev([1.0, -1.0]))
    assert info["status"] == ppcg.BREAKDOWN


# ---------------------------------------------------------------- FP32 inner solves

@pytest.mark.parametrize("gen", [lambda: stencil27_lognormal(16, seed=1), lambda: poisson3d(24),
                                 lambda: random_spd(20000, seed=3), lambda: shifted(poisson2d(90), 0.01)])
def test_pcg_fp32_inner_reaches_fp64_tolerance(gen):
    """Algorithm 1 in FP32 (values, vectors) with FP64 reliable updates: the
    FP64 iterate meets the FP64 tolerance on the FP64 operator, and since the
    direction is kept across the updates (no restart of the Krylov sequence)
    the iteration count stays close to FP64 Algorithm 1's."""
    A = gen()
    b = problem(A)
    x, info = Solver(A, tol=1e-10, method="pcg", precision="mixed").solve(dev(b))
    assert info["status"] == ppcg.OK, info
    assert info["outer_iters"] >= 2, info  # at 1e-2 per stretch, 1e-10 takes several
    assert info["rel_resid_true"] <= 1e-10
    assert oracle.true_relres(A, b, host(x)) <= 1e-10
    ref = oracle.pcg(A, b, tol=1e-10)
    assert info["iters"] <= 1.15 * ref.iters + 5, (info["iters"], ref.iters)
    assert relerr(host(x), ref.x) <= 1e-5


@pytest.mark.parametrize("gen", [lambda: poisson3d(24), lambda: stencil27_lognormal(14, seed=2),
                                 lambda: random_spd(5000, seed=6)])
def test_pcg_fp32_first_inner_solve_follows_algorithm1(gen):
    """One stretch: from x0 = 0 the FP32 sequence is Algorithm 1 on
    b / ||b||, and x = ||b|| x32 at its first pause.  After its k iterations x agrees
    with the oracle's k iterations of Algorithm 1 in FP64 to FP32 accuracy;
    a wrong step (a sign, a dropped term, a stale direction) misses by O(1)."""
    A = gen()
    b = problem(A)
    x, info = Solver(A, tol=1e-10, method="pcg", precision="mixed", inner_tol=0.1, max_outer=1).solve(dev(b))
    assert info["status"] == ppcg.NOT_CONVERGED and info["outer_iters"] == 1, info
    k = info["iters"]
    assert k >= 2
    ref = oracle.pcg(A, b, fixed_iters=k)
    assert relerr(host(x), ref.x) <= 1e-4, (k, relerr(host(x), ref.x))
    # the inner stop: relative recurrence residual below 0.1 after k, not k - 1
    prev = oracle.pcg(A, b, fixed_iters=k - 1)
    assert oracle.true_relres(A, b, prev.x) > 0.05


def test_pcg_fp32_inner_batch_bitwise_equals_solo():
    mats = [stencil27_lognormal(12, seed=4), shifted(poisson2d(70), 0.01), random_spd(4000, seed=2)]
    bs = [problem(A, seed=80 + i) for i, A in enumerate(mats)]
    kw = dict(tol=1e-10, method="pcg", precision="mixed")
    solo = [host(Solver(A, **kw).solve(dev(b))[0]) for A, b in zip(mats, bs)]
    xs, infos = solve_batch([Solver(A, **kw) for A in mats], [dev(b) for b in bs])
    for x, xs_, info in zip(xs, solo, infos):
        assert np.array_equal(host(x), xs_)
        assert info["status"] == ppcg.OK and info["rel_resid_true"] <= 1e-10


def test_pcg_fp32_inner_csr_vector_matches_tolerance():
    A = random_spd(6000, seed=9)
    b = problem(A)
    x, info = Solver(A, tol=1e-10, method="pcg", precision="mixed", spmv_format="csr_vector").solve(dev(b))
    assert info["status"] == ppcg.OK and info["rel_resid_true"] <= 1e-10
    assert oracle.true_relres(A, b, host(x)) <= 1e-10


# ---------------------------------------------------------------- FP32 matrix values

def _round32(A):
    return CSR(A.n, A.rp, A.ci, A.val.astype(np.float32).astype(np.float64), A.name + "_fp32")


def _diag_fp32_exact(A):
    """A with its diagonal rounded to FP32, so that the Jacobi preconditioner
    of A and of its FP32 rounding coincide (still SPD: the change is ~1e-7
    relative)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    val = A.val.copy()
    on = A.ci == rows
    val[on] = val[on].astype(np.float32).astype(np.float64)
    return CSR(A.n, A.rp, A.ci, val, A.name)


@pytest.mark.parametrize("gen", [lambda: stencil27_lognormal(14, seed=2), lambda: random_spd(5000, seed=6)])
def test_pcg_fp32_values_iterates_match_oracle_on_rounded_matrix(gen):
    """Until the first reliable update the iteration is Algorithm 1 on the
    FP32-rounded operator with FP64 vectors and accumulation; x0 = 0 makes the
    initial residual b either way, so the oracle on the rounded matrix is the
    reference."""
    A = _diag_fp32_exact(gen())
    b = problem(A)
    S = Solver(A, method="pcg", precision="mixed_values", inner_tol=1e-30, spmv_format="sell")
    for k in (1, 4, 13):
        S.set_options(method="pcg", precision="mixed_values", fixed_iters=k, inner_tol=1e-30)
        x, info = S.solve(dev(b))
        ref = oracle.pcg(_round32(A), b, fixed_iters=k)
        assert info["iters"] == k and info["outer_iters"] == 0
        assert relerr(host(x), ref.x) <= 1e-10, k


@pytest.mark.parametrize("gen,factor", [(lambda: stencil27_lognormal(16, seed=1), 1e-3),
                                        (lambda: stencil27_lognormal(16, seed=1), 0.3),
                                        (lambda: poisson3d(24), 1e-2),
                                        (lambda: random_spd(20000, seed=3), 1e-3)])
def test_pcg_fp32_values_reliable_updates_reach_fp64_tolerance(gen, factor):
    A = gen()
    b = problem(A)
    x, info = Solver(A, tol=1e-10, method="pcg", precision="mixed_values", inner_tol=factor).solve(dev(b))
    ref = oracle.pcg(A, b, tol=1e-10)
    assert info["status"] == ppcg.OK, info
    assert info["rel_resid_true"] <= 1e-10
    assert oracle.true_relres(A, b, host(x)) <= 1e-10
    assert info["iters"] <= 1.15 * ref.iters + 5, (info["iters"], ref.iters)
    assert relerr(host(x), ref.x) <= 1e-5


def test_pcg_fp32_values_batch_bitwise_equals_solo():
    mats = [stencil27_lognormal(12, seed=4), shifted(poisson2d(70), 0.01), random_spd(4000, seed=2)]
    bs = [problem(A, seed=70 + i) for i, A in enumerate(mats)]
    kw = dict(tol=1e-10, method="pcg", precision="mixed_values")
    solo = [host(Solver(A, **kw).solve(dev(b))[0]) for A, b in zip(mats, bs)]
    xs, infos = solve_batch([Solver(A, **kw) for A in mats], [dev(b) for b in bs])
    for x, xs_, info in zip(xs, solo, infos):
        assert np.array_equal(host(x), xs_)
        assert info["status"] == ppcg.OK and info["rel_resid_true"] <= 1e-10


def test_pcg_batch_bitwise_equals_solo():
    mats = [poisson2d(40), shifted(poisson2d(53), 0.3), random_spd(2500, seed=8), stencil27_lognormal(10, seed=2),
            poisson3d(20)]
    bs = [problem(A, seed=60 + i) for i, A in enumerate(mats)]
    solo = [Solver(A, tol=1e-10, method="pcg").solve(dev(b)) for A, b in zip(mats, bs)]
    xs, infos = solve_batch([Solver(A, tol=1e-10, method="pcg") for A in mats], [dev(b) for b in bs])
    for (xs_, is_), x, info, A, b in zip(solo, xs, infos, mats, bs):
        assert np.array_equal(host(x), host(xs_)), A.name
        assert info["iters"] == is_["iters"]
        assert info["status"] == ppcg.OK
        assert abs(info["iters"] - oracle.pcg(A, b, tol=1e-10).iters) <= 2


def test_pcg_kernel_timing():
    A = poisson3d(40)
    S = Solver(A, method="pcg")
    ms_vma, ms_spmv = S.time_kernels(dev(problem(A)), 20)
    assert ms_vma > 0 and ms_spmv > 0
