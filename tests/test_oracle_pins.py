"""Pins of the FP64 oracle to facts fixed outside it.

Each test ties the oracle (Algorithms 1 and 2 of Tiwari & Vadhiyar, Section
III, with the Jacobi preconditioner of Section V-A) to something it does not
compute itself: exact rational solutions, the Galerkin characterisation of CG
iterates, dense Cholesky, closed-form Poisson eigenpairs, finite termination
(CG solves an N x N SPD system in N steps in exact arithmetic, Section I),
the symmetric Jacobi scaling identity, and the printed sizes of Table 2.
A dropped term, a wrong sign or index, or a transposed operand in either
algorithm breaks at least one of them.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import (CSR, nnz_poisson125, nnz_poisson2d, nnz_poisson3d, nnz_stencil27, poisson125,
                       poisson2d, poisson2d_eigpair, poisson3d, poisson3d_eigpair, random_spd,
                       rhs_from_solution, stencil27_lognormal, xstar_uniform)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def tiny_spd(n: int, seed: int) -> CSR:
    """Small SPD matrix with integer entries (exact in FP64 and in Fractions)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < 0.6:
                v = int(rng.integers(-3, 4))
                A[i, j] = A[j, i] = v
    for i in range(n):
        A[i, i] = int(np.abs(A[i]).sum()) + int(rng.integers(1, 6))
    return dense_to_csr(A.astype(np.float64))


def dense_to_csr(D: np.ndarray) -> CSR:
    n = D.shape[0]
    rp, ci, val = [0], [], []
    for i in range(n):
        for j in range(n):
            if D[i, j] != 0 or i == j:
                ci.append(j)
                val.append(D[i, j])
        rp.append(len(ci))
    return CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(val, np.float64))


def frac_solve(M, rhs):
    """Gaussian elimination in exact rational arithmetic."""
    n = len(M)
    a = [[Fraction(M[i][j]) for j in range(n)] + [Fraction(rhs[i])] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c] / a[c][c]
                a[r] = [x - f * y for x, y in zip(a[r], a[c])]
    return [a[i][n] / a[i][i] for i in range(n)]


def galerkin_iterate(D: np.ndarray, b, k: int):
    """x_k of Jacobi-PCG from x0 = 0, from its characterisation, exactly.

    x_k is the unique point of the Krylov space span{z, (M^-1 A) z, ...,
    (M^-1 A)^{k-1} z}, z = M^-1 b, whose residual is orthogonal to that space
    (equivalently, it minimises the A-norm of the error over the space).
    """
    n = D.shape[0]
    A = [[Fraction(int(D[i, j])) for j in range(n)] for i in range(n)]
    dinv = [1 / A[i][i] for i in range(n)]
    bb = [Fraction(int(v)) for v in b]
    basis = [[dinv[i] * bb[i] for i in range(n)]]
    for _ in range(1, k):
        v = basis[-1]
        Av = [sum(A[i][j] * v[j] for j in range(n)) for i in range(n)]
        basis.append([dinv[i] * Av[i] for i in range(n)])
    AV = [[sum(A[i][j] * v[j] for j in range(n)) for i in range(n)] for v in basis]
    G = [[sum(basis[a][i] * AV[c][i] for i in range(n)) for c in range(k)] for a in range(k)]
    rhs = [sum(basis[a][i] * bb[i] for i in range(n)) for a in range(k)]
    try:
        y = frac_solve(G, rhs)
    except StopIteration:  # Krylov space became invariant: x_k = x_{k-1} = A^-1 b
        return galerkin_iterate(D, b, k - 1)
    return np.array([float(sum(y[a] * basis[a][i] for a in range(k))) for i in range(n)])


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- SpMV and generators

@pytest.mark.parametrize("n,jk", [(9, (1, 1)), (9, (2, 5)), (16, (3, 7)), (16, (16, 1))])
def test_spmv_poisson2d_eigpairs(n, jk):
    A = poisson2d(n)
    lam, v = poisson2d_eigpair(n, *jk)
    assert np.abs(oracle.spmv(A, v) - lam * v).max() <= 1e-14 * 8


@pytest.mark.parametrize("n,jkl", [(6, (1, 1, 1)), (7, (2, 3, 5)), (8, (8, 1, 4))])
def test_spmv_poisson3d_eigpairs(n, jkl):
    A = poisson3d(n)
    lam, v = poisson3d_eigpair(n, *jkl)
    assert np.abs(oracle.spmv(A, v) - lam * v).max() <= 1e-14 * 12


def test_spmv_brute_force_dense():
    A = random_spd(60, seed=3)
    x = xstar_uniform(60, seed=4)
    D = A.dense()
    exact = [math.fsum(D[i, j] * x[j] for j in range(60)) for i in range(60)]
    assert np.allclose(oracle.spmv(A, x), exact, rtol=0, atol=1e-14)


@pytest.mark.parametrize("gen,shift", [(lambda: stencil27_lognormal(7, seed=2), 1e-3),
                                       (lambda: random_spd(400, seed=5), 1e-2)])
def test_graph_laplacian_constant_mode(gen, shift):
    """A = L + shift*I with L a graph Laplacian, so A 1 = shift 1."""
    A = gen()
    y = oracle.spmv(A, np.ones(A.n))
    scale = np.abs(A.val).max()
    assert np.abs(y - shift).max() <= 64 * np.finfo(float).eps * scale


def test_nnz_formulas():
    for n in (2, 3, 8, 31):
        assert poisson2d(n).nnz == nnz_poisson2d(n)
    for n in (2, 3, 9):
        assert poisson3d(n).nnz == nnz_poisson3d(n)
        assert stencil27_lognormal(n).nnz == nnz_stencil27(n)
        assert poisson125(n).nnz == nnz_poisson125(n)


def test_table2_sizes_match_125pt_formula():
    rows = []
    with open(os.path.join(GOLDEN, "table2_poisson125.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, N, nnz = line.split()
                rows.append((name, int(N), int(nnz)))
    assert len(rows) == 4
    for name, N, nnz in rows:
        side = round(N ** (1 / 3))
        assert side ** 3 == N, name
        assert nnz_poisson125(side) == nnz, name


def test_generators_symmetric_with_diagonal():
    for A in (poisson2d(7), poisson3d(5), stencil27_lognormal(4, seed=1), random_spd(300, seed=2),
              poisson125(6)):
        S = A.to_scipy()
        assert abs(S - S.T).max() == 0
        assert np.all(A.diag() > 0)
        for i in range(A.n):
            cols = A.ci[A.rp[i]:A.rp[i + 1]]
            assert np.all(np.diff(cols) > 0)


# ---------------------------------------------------------------- Jacobi

def test_jacobi_is_inverse_diagonal():
    A = stencil27_lognormal(5, seed=4)
    d = oracle.jacobi(A)
    assert np.array_equal(d, 1.0 / A.diag())


def test_jacobi_rejects_bad_diagonal():
    D = np.array([[2.0, -1.0], [-1.0, 0.0]])
    with pytest.raises(ValueError):
        oracle.jacobi(dense_to_csr(D))
    r = oracle.pipecg(dense_to_csr(D), np.ones(2))
    assert r.status == oracle.BAD_INPUT


@pytest.mark.parametrize("solver", [oracle.pcg, oracle.pipecg])
def test_jacobi_symmetric_scaling_identity(solver):
    """Jacobi-PCG on A equals plain CG on D^-1/2 A D^-1/2 (unit diagonal, so
    its Jacobi preconditioner is the identity) after x = D^-1/2 y."""
    A = stencil27_lognormal(6, seed=7, shift=0.5)  # well conditioned: rounding stays small
    d = A.diag()
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    As = CSR(A.n, A.rp, A.ci, A.val / np.sqrt(d[rows] * d[A.ci]))
    b = rhs_from_solution(A, xstar_uniform(A.n, 8))
    bs = b / np.sqrt(d)
    for k in (3, 12, 30):
        x = solver(A, b, fixed_iters=k).x
        y = solver(As, bs, fixed_iters=k).x
        assert relerr(x, y / np.sqrt(d)) <= 1e-10, k


# ---------------------------------------------------------------- exact arithmetic pins

@pytest.mark.parametrize("dots", ["seq", "comp"])
@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("solver", [oracle.pcg, oracle.pipecg])
def test_iterates_match_exact_galerkin(seed, solver, dots):
    n = 4 + seed % 4
    A = tiny_spd(n, seed)
    D = A.dense()
    b = np.random.default_rng(100 + seed).integers(-5, 6, size=n).astype(np.float64)
    b[0] = 7.0
    for k in range(1, n + 1):
        exact = galerkin_iterate(D, b, k)
        got = solver(A, b, fixed_iters=k, dots=dots).x
        assert relerr(got, exact) <= 1e-11, (k, relerr(got, exact))


# ---------------------------------------------------------------- dot products

def test_compensated_dot_recovers_cancelled_terms():
    """1 + 1e100 + 1 - 1e100 = 2: summed left to right the two ones are lost
    (0); the compensated sum keeps them."""
    a = np.array([1.0, 1e100, 1.0, -1e100])
    assert oracle.dot(a, np.ones(4)) == 0.0
    assert oracle.dot(a, np.ones(4), dots="comp") == 2.0


@pytest.mark.parametrize("seed", range(4))
def test_dot_error_bounds_against_exact_sum(seed):
    """Products of small integers times powers of two are exact in FP64, so
    the exact dot product is a rational sum.  Left to right the error is at
    most (n-1) eps sum|a_i b_i| (the textbook bound); compensated (Neumaier)
    it is at most eps |sum| + 2 n eps^2 sum|a_i b_i|."""
    rng = np.random.default_rng(seed)
    n = 2000
    a = rng.integers(-2 ** 20, 2 ** 20, size=n) * np.exp2(rng.integers(-40, 40, size=n))
    b = rng.integers(-2 ** 20, 2 ** 20, size=n) * np.exp2(rng.integers(-40, 40, size=n))
    exact = sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b))
    mag = float(sum(abs(Fraction(float(x)) * Fraction(float(y))) for x, y in zip(a, b)))
    eps = np.finfo(float).eps / 2
    seq = oracle.dot(a, b)
    comp = oracle.dot(a, b, dots="comp")
    assert abs(Fraction(seq) - exact) <= (n - 1) * eps * mag
    assert abs(Fraction(comp) - exact) <= eps * abs(float(exact)) + 2 * n * eps * eps * mag
    # the bound is far tighter than the sequential one: the sums differ
    assert abs(Fraction(comp) - exact) <= abs(Fraction(seq) - exact)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("solver", [oracle.pcg, oracle.pipecg])
def test_finite_termination_exact_solution(seed, solver):
    n = 4 + seed % 4
    A = tiny_spd(n, 50 + seed)
    D = A.dense()
    b = np.random.default_rng(seed).integers(-9, 10, size=n).astype(np.float64)
    b[-1] = 3.0
    exact = np.array([float(v) for v in frac_solve(D.astype(int).tolist(), b.astype(int).tolist())])
    r = solver(A, b, tol=1e-12)
    assert r.status == oracle.OK
    assert r.iters <= n
    assert relerr(r.x, exact) <= 1e-12


@pytest.mark.parametrize("gen", [lambda: random_spd(200, seed=11), lambda: poisson2d(12),
                                 lambda: stencil27_lognormal(5, seed=3)])
def test_solution_matches_dense_cholesky(gen):
    A = gen()
    D = A.dense()
    b = np.random.default_rng(9).uniform(-1, 1, size=A.n)
    L = np.linalg.cholesky(D)
    xc = np.linalg.solve(L.T, np.linalg.solve(L, b))
    ev = np.linalg.eigvalsh(D)
    kappa = ev[-1] / ev[0]
    for solver in (oracle.pcg, oracle.pipecg):
        r = solver(A, b, tol=1e-11)
        assert r.status == oracle.OK
        assert relerr(r.x, xc) <= 10 * kappa * 1e-11


def test_eigenvector_rhs_converges_in_one_iteration():
    n = 10
    A = poisson2d(n)
    lam, v = poisson2d_eigpair(n, 3, 4)
    r = oracle.pipecg(A, v, tol=1e-12)
    assert r.iters == 1
    assert relerr(r.x, v / lam) <= 1e-14


def test_k_distinct_eigencomponents_take_k_iterations():
    n = 12
    A = poisson2d(n)
    modes = [(1, 1), (1, 2), (2, 2), (1, 4), (3, 5)]
    lams = []
    b = np.zeros(A.n)
    for c, (j, k) in enumerate(modes):
        lam, v = poisson2d_eigpair(n, j, k)
        lams.append(lam)
        b += (c + 1) * v
    assert len(set(np.round(lams, 12))) == len(modes)
    for solver in (oracle.pcg, oracle.pipecg):
        r = solver(A, b, tol=1e-10)
        assert r.status == oracle.OK
        assert r.iters == len(modes)


# ---------------------------------------------------------------- PCG vs PIPECG, invariants

@pytest.mark.parametrize("gen,kb", [(lambda: poisson2d(64), ((10, 1e-12), (50, 1e-11), (100, 1e-10))),
                                    (lambda: random_spd(3000, seed=1), ((10, 1e-12), (40, 1e-11))),
                                    # ill conditioned (shift 1e-3): rounding differences between the
                                    # two recurrences grow with k
                                    (lambda: stencil27_lognormal(10, seed=1), ((10, 1e-10), (50, 1e-7)))])
def test_pcg_and_pipecg_iterates_agree(gen, kb):
    """Same iterates in exact arithmetic; in FP64 they agree to rounding."""
    A = gen()
    b = rhs_from_solution(A, xstar_uniform(A.n))
    for k, bound in kb:
        a = oracle.pcg(A, b, fixed_iters=k).x
        c = oracle.pipecg(A, b, fixed_iters=k).x
        assert relerr(c, a) <= bound, k


@pytest.mark.parametrize("gen", [lambda: random_spd(300, seed=4), lambda: poisson3d(8)])
def test_pipecg_recurrence_invariants(gen):
    """In exact arithmetic w = A u, s = A p, q = M^-1 s, z = A q, m = M^-1 w,
    n = A m, and (p, A p) = gamma_{i-1} / alpha_{i-1}."""
    A = gen()
    b = rhs_from_solution(A, xstar_uniform(A.n, 3))
    dinv = 1.0 / A.diag()
    S = A.to_scipy()
    first = oracle.pipecg(A, b, fixed_iters=1, state=True).state
    scale = {k: np.linalg.norm(v) for k, v in first.items() if isinstance(v, np.ndarray)}
    scale["r"] = np.linalg.norm(b)
    pap_first = float(first["p"] @ (S @ first["p"]))

    def drift(a, b_, name):  # relative to the vector's size at the first iteration
        return float(np.linalg.norm(a - b_) / scale[name])

    for k in (1, 5, 20, 40):
        st = oracle.pipecg(A, b, fixed_iters=k, state=True).state
        assert drift(S @ st["u"], st["w"], "w") <= 1e-12
        assert drift(S @ st["p"], st["s"], "s") <= 1e-12
        assert drift(dinv * st["s"], st["q"], "q") <= 1e-12
        assert drift(S @ st["q"], st["z"], "z") <= 1e-12
        assert np.array_equal(dinv * st["w"], st["m"])
        assert np.array_equal(oracle.spmv(A, st["m"]), st["n"])
        pap = float(st["p"] @ (S @ st["p"]))
        assert abs(pap - st["gamma_prev"] / st["alpha_prev"]) <= 1e-10 * pap_first
        assert drift(b - S @ st["x"], st["r"], "r") <= 1e-12


def test_residuals_mutually_orthogonal():
    """(r_i, u_j) = 0 for i != j (M-orthogonality of the residuals)."""
    A = random_spd(200, seed=8)
    b = rhs_from_solution(A, xstar_uniform(A.n, 2))
    R, U = [], []
    for k in range(6):
        st = oracle.pipecg(A, b, fixed_iters=k, state=True).state if k else None
        if k == 0:
            r0 = b.copy()
            R.append(r0)
            U.append(r0 / A.diag())
        else:
            R.append(st["r"])
            U.append(st["u"])
    for i in range(6):
        for j in range(6):
            if i != j:
                c = abs(R[i] @ U[j]) / (np.linalg.norm(R[i]) * np.linalg.norm(U[j]))
                assert c <= 1e-10


def test_iteration_count_within_cg_bound_c1():
    """2-D 64x64 Poisson: kappa from the closed-form extreme eigenvalues and the
    classical CG bound on the iterations for a 1e-8 reduction."""
    n = 64
    A = poisson2d(n)
    lmin = poisson2d_eigpair(n, 1, 1)[0]
    lmax = poisson2d_eigpair(n, n, n)[0]
    kappa = lmax / lmin
    eps = 1e-8
    bound = math.ceil(math.log(2 * math.sqrt(kappa) / eps) /
                      math.log((math.sqrt(kappa) + 1) / (math.sqrt(kappa) - 1)))
    b = rhs_from_solution(A, xstar_uniform(A.n))
    r = oracle.pipecg(A, b, tol=eps)
    assert r.status == oracle.OK
    assert r.rel_true <= eps
    assert 0 < r.iters <= bound


# ---------------------------------------------------------------- stopping and failure semantics

def test_maxit_zero_and_tol_zero():
    A = poisson2d(8)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    r = oracle.pipecg(A, b, maxit=0)
    assert r.iters == 0 and r.status == oracle.NOT_CONVERGED and np.all(r.x == 0)
    r = oracle.pipecg(A, b, tol=0.0, maxit=25)
    assert r.iters == 25 and r.status in (oracle.NOT_CONVERGED, oracle.BREAKDOWN)


def test_converged_initial_guess_and_zero_rhs():
    A = poisson2d(8)
    xs = xstar_uniform(A.n)
    b = oracle.spmv(A, xs)
    r = oracle.pipecg(A, b, x0=xs, tol=1e-12)
    assert r.iters == 0 and r.status == oracle.OK and np.array_equal(r.x, xs)
    r = oracle.pipecg(A, np.zeros(A.n), tol=1e-8)
    assert r.iters == 0 and r.status == oracle.OK and np.all(r.x == 0)


def test_absolute_and_relative_modes_coincide_for_constant_diagonal():
    """With diag(A) = d I, u = r / d, so sqrt((u,u)) < t  <=>  ||r|| < d t."""
    A = poisson3d(10)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    tol = 1e-7
    rel = oracle.pipecg(A, b, tol=tol, history=True)
    bn = np.linalg.norm(b)
    abs_tol = tol * bn / 6.0 * (1 + 1e-9)
    ab = oracle.pipecg(A, b, tol=abs_tol, stop=oracle.STOP_ABS, history=True)
    assert abs(ab.iters - rel.iters) <= 1
    assert np.allclose(ab.hist[:5] * 6.0, rel.hist[:5], rtol=1e-12)


def test_breakdown_on_indefinite_matrix():
    D = np.array([[1.0, 2.0], [2.0, 1.0]])  # eigenvalues 3 and -1, positive diagonal
    b = np.array([1.0, -1.0])  # eigenvector of -1
    for solver in (oracle.pcg, oracle.pipecg):
        r = solver(dense_to_csr(D), b)
        assert r.status == oracle.BREAKDOWN
        assert r.iters == 0


def test_fixed_iterations_ignore_tolerance():
    A = poisson2d(16)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    r = oracle.pipecg(A, b, tol=1.0, fixed_iters=7)
    assert r.iters == 7


def test_restart_from_true_residual():
    """An unreachable tolerance makes the recurrence residual drop below it
    while the true residual stalls: the solver restarts, then stagnates."""
    A = stencil27_lognormal(8, seed=2)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    for solver in (oracle.pcg, oracle.pipecg):
        r = solver(A, b, tol=1e-18, maxit=5000, max_restarts=2)
        assert r.status in (oracle.STAGNATED, oracle.BREAKDOWN)
        assert r.restarts == 2
        assert r.rel_true <= 1e-10


def test_breakdown_near_convergence_restarts_pipecg():
    """Pipelined CG loses its recurrences near its attainable accuracy; the
    breakdown then restarts the method from x instead of failing."""
    A = stencil27_lognormal(8, seed=2)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    r0 = oracle.pipecg(A, b, tol=1e-14, maxit=5000, max_restarts=0)
    r3 = oracle.pipecg(A, b, tol=1e-14, maxit=5000, max_restarts=3)
    assert r0.status == oracle.BREAKDOWN
    assert r3.restarts >= 1
    assert r3.rel_true < r0.rel_true
