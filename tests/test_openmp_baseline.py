"""PIPECG-OpenMP, the paper's CPU baseline (Sections V-A, V-B: Algorithm 2 on
host threads with the vector-update loops merged), is a timing build: these
CPU tests hold it to the sequential oracle.  With one thread its sums run in
the oracle's order, so it is bitwise equal; with several, the reductions are
associated per thread, and fixed iterates stay within the 1e-10 bar."""

import numpy as np
import pytest

import oracle
from workloads import poisson2d, poisson3d, random_spd, rhs_from_solution, stencil27_lognormal, xstar_uniform

CASES = [(lambda: poisson3d(24), 40), (lambda: stencil27_lognormal(12, seed=3), 30),
         (lambda: random_spd(5000, seed=1), 25), (lambda: poisson2d(37), 60)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_one_thread_is_the_oracle(case):
    gen, k = CASES[case]
    A = gen()
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    x, st, it = oracle.pipecg_openmp(A, b, fixed_iters=k, threads=1)
    ref = oracle.pipecg(A, b, fixed_iters=k)
    assert st == oracle.OK and it == k
    assert np.array_equal(x, ref.x)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_threads_within_rounding(case):
    gen, k = CASES[case]
    A = gen()
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    x, st, it = oracle.pipecg_openmp(A, b, fixed_iters=k, threads=4)
    ref = oracle.pipecg(A, b, fixed_iters=k)
    assert st == oracle.OK and it == k
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-10


def test_tolerance_solve_and_paper_stop():
    A = poisson3d(20)
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    x, st, it = oracle.pipecg_openmp(A, b, tol=1e-10, threads=4)
    ref = oracle.pipecg(A, b, tol=1e-10)
    assert st == oracle.OK and abs(it - ref.iters) <= 2
    assert oracle.true_relres(A, b, x) <= 1e-10
    bp = rhs_from_solution(A, np.full(A.n, 1 / np.sqrt(A.n)))
    x, st, it = oracle.pipecg_openmp(A, bp, tol=1e-5, stop=oracle.STOP_ABS, threads=3)
    ref = oracle.pipecg(A, bp, tol=1e-5, stop=oracle.STOP_ABS)
    assert st == oracle.OK and abs(it - ref.iters) <= 2
