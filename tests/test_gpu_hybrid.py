"""Host cores + GPU together (Section IV-C, Hybrid-PIPECG-3): Algorithm 2 with
the rows split between host threads and the GPU, checked against the oracle's
Algorithm 2.  Each side sums its SpMV rows in stored column order (part 1
then part 2 added), the dot products are split between the sides and added on
the host, so iterates match the oracle to rounding: 1e-10 relative after fixed
iteration counts, iteration counts within 2 for tolerance solves."""

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Hybrid, PPCGError
from workloads import (poisson2d, poisson3d, random_spd, rhs_from_solution, stencil27_lognormal, xstar_paper,
                       xstar_uniform)

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(A, seed=1):
    return rhs_from_solution(A, xstar_uniform(A.n, seed))


CASES = {
    "poisson2d_37": lambda: poisson2d(37),
    "poisson3d_24": lambda: poisson3d(24),
    "random_spd_3001": lambda: random_spd(3001, seed=2),
    "stencil27_12": lambda: stencil27_lognormal(12, seed=3),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("share", [0.3, 0.5, 0.9])
def test_hybrid_fixed_iterates_match_oracle(name, share):
    A = CASES[name]()
    b = problem(A)
    for k in (1, 7, 30):
        H = Hybrid(A, host_threads=3, cpu_share=share, fixed_iters=k)
        info_h = H.info()
        assert 0 < info_h["n_cpu"] < A.n and info_h["n_cpu"] + info_h["n_gpu"] == A.n
        x, info = H.solve(b)
        ref = oracle.pipecg(A, b, fixed_iters=k)
        assert info["status"] == ppcg.OK and info["iters"] == k == ref.iters
        assert relerr(x, ref.x) <= 1e-10, (k, relerr(x, ref.x))
        H.close()


@pytest.mark.parametrize("name,tol", [("poisson3d_24", 1e-10), ("random_spd_3001", 1e-10), ("stencil27_12", 1e-8)])
def test_hybrid_tolerance_solve(name, tol):
    A = CASES[name]()
    b = problem(A)
    x, info = Hybrid(A, host_threads=4, cpu_share=0.4, tol=tol).solve(b)
    ref = oracle.pipecg(A, b, tol=tol)
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - ref.iters) <= 2
    assert info["rel_resid_true"] <= tol
    assert oracle.true_relres(A, b, x) <= tol


def test_hybrid_degenerate_splits_and_initial_guess():
    A = poisson2d(30)
    b = problem(A)
    ref = oracle.pipecg(A, b, fixed_iters=20)
    for share in (0.0, 1.0):
        x, info = Hybrid(A, host_threads=2, cpu_share=share, fixed_iters=20).solve(b)
        assert relerr(x, ref.x) <= 1e-10
    x0 = xstar_uniform(A.n, 9)
    x, info = Hybrid(A, host_threads=2, cpu_share=0.5, fixed_iters=20).solve(b, x0)
    assert relerr(x, oracle.pipecg(A, b, x0=x0, fixed_iters=20).x) <= 1e-10


def test_hybrid_performance_model_split():
    A = poisson3d(40)
    b = problem(A)
    H = Hybrid(A, host_threads=4, tol=1e-8)
    i = H.info()
    assert i["t_cpu_spmv_ms"] > 0 and i["t_gpu_spmv_ms"] > 0
    assert i["n_cpu"] + i["n_gpu"] == A.n
    # the host takes at most its share of the non-zeros (Section IV-C)
    r_cpu = (1 / i["t_cpu_spmv_ms"]) / (1 / i["t_cpu_spmv_ms"] + 1 / i["t_gpu_spmv_ms"])
    assert A.rp[i["n_cpu"]] <= A.nnz * r_cpu * (1 + 1e-9)
    assert i["nnz_cpu_local"] + i["nnz_cpu_remote"] == A.rp[i["n_cpu"]]
    x, info = H.solve(b)
    assert info["status"] == ppcg.OK and oracle.true_relres(A, b, x) <= 1e-8


def test_hybrid_paper_protocol():
    A = poisson3d(32)
    b = rhs_from_solution(A, xstar_paper(A.n))
    x, info = Hybrid(A, host_threads=4, cpu_share=0.25, tol=1e-5, stop="abs", max_iter=10000).solve(b)
    ref = oracle.pipecg(A, b, tol=1e-5, stop=oracle.STOP_ABS, maxit=10000)
    assert info["status"] == ppcg.OK and abs(info["iters"] - ref.iters) <= 2
    assert info["precond_norm"] < 1e-5


# ---------------------------------------------------------------- task-parallel schemes

@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("name", sorted(CASES))
def test_task_schemes_fixed_iterates_match_oracle(scheme, name):
    """Hybrid-1 (w, r, u copied, dots on the host) and Hybrid-2 (n copied, the
    host repeats the updates of z, q, s, r, u, w, m): the GPU runs every
    update and the SpMV with Algorithm 2's arithmetic, the host sums the dot
    products in a fixed thread order, so iterates match the oracle to 1e-10."""
    A = CASES[name]()
    b = problem(A)
    for k in (1, 7, 30):
        H = Hybrid(A, host_threads=3, scheme=scheme, fixed_iters=k)
        i = H.info()
        assert i["scheme"] == scheme and i["n_cpu"] == 0 and i["n_gpu"] == A.n
        assert i["copy_bytes_per_iter"] == (3 if scheme == 1 else 1) * 8.0 * A.n
        x, info = H.solve(b)
        ref = oracle.pipecg(A, b, fixed_iters=k)
        assert info["status"] == ppcg.OK and info["iters"] == k == ref.iters
        assert relerr(x, ref.x) <= 1e-10, (k, relerr(x, ref.x))
        H.close()


@pytest.mark.parametrize("scheme", [1, 2])
def test_task_schemes_tolerance_solve_and_initial_guess(scheme):
    A = poisson3d(24)
    b = problem(A)
    x, info = Hybrid(A, host_threads=4, scheme=scheme, tol=1e-10).solve(b)
    ref = oracle.pipecg(A, b, tol=1e-10)
    assert info["status"] == ppcg.OK and abs(info["iters"] - ref.iters) <= 2
    assert info["rel_resid_true"] <= 1e-10 and oracle.true_relres(A, b, x) <= 1e-10
    x0 = xstar_uniform(A.n, 9)
    x, info = Hybrid(A, host_threads=2, scheme=scheme, fixed_iters=20).solve(b, x0)
    assert relerr(x, oracle.pipecg(A, b, x0=x0, fixed_iters=20).x) <= 1e-10
    # the paper's absolute stop on the preconditioned residual
    P = poisson3d(20)
    bp = rhs_from_solution(P, xstar_paper(P.n))
    x, info = Hybrid(P, host_threads=2, scheme=scheme, tol=1e-5, stop="abs", max_iter=10000).solve(bp)
    refp = oracle.pipecg(P, bp, tol=1e-5, stop=oracle.STOP_ABS, maxit=10000)
    assert info["status"] == ppcg.OK and abs(info["iters"] - refp.iters) <= 2


def test_task_schemes_agree_with_each_other():
    """Both task schemes form the same iteration on the GPU; Hybrid-2's host
    copies are the GPU's bit for bit and its dot products are summed as
    Hybrid-1 sums the copied vectors', so the two give the same x."""
    A = stencil27_lognormal(14, seed=5)
    b = problem(A)
    x1, i1 = Hybrid(A, host_threads=3, scheme=1, fixed_iters=40).solve(b)
    x2, i2 = Hybrid(A, host_threads=3, scheme=2, fixed_iters=40).solve(b)
    assert np.array_equal(x1, x2)


def test_hybrid_rejects_unsupported_options():
    A = poisson2d(8)
    with pytest.raises(PPCGError):
        Hybrid(A, precision="mixed_values")
    with pytest.raises(PPCGError):
        Hybrid(A, vec_mem="device")
    with pytest.raises(PPCGError):
        Hybrid(A, cpu_share=1.5)
    with pytest.raises(PPCGError):
        Hybrid(A, scheme=1, cpu_share=0.5)  # every row is on the GPU in the task schemes
    with pytest.raises(PPCGError):
        Hybrid(A, scheme=4)
