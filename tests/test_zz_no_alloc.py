"""ppcg_solve_noalloc (the entry point that allocates nothing) against
ppcg_solve on a handle with the CSR-vector SpMV, through the C ABI.

Both run the same kernels in the same order on the same tiles, so the
results must be bitwise equal (stronger than the 1e-10 parity bar).  Two
calls in a row share the static scratch array: the second, smaller system
must not see the first one's leftovers.  Sizes above the array's limit are
rejected with an argument error and x untouched.
"""

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Solver, solve_noalloc
from workloads import poisson2d, poisson3d, random_spd, rhs_from_solution, stencil27_lognormal, xstar_uniform

pytestmark = pytest.mark.gpu

MAX_ROWS = 1 << 19


def _dev_csr(A):
    import torch

    return (torch.as_tensor(np.ascontiguousarray(A.rp, np.int32)).cuda(),
            torch.as_tensor(np.ascontiguousarray(A.ci, np.int32)).cuda(),
            torch.as_tensor(np.ascontiguousarray(A.val, np.float64)).cuda())


def _pair(A, b, **opts):
    """(x, info) from ppcg_solve_noalloc and from ppcg_solve (CSR-vector)."""
    import torch

    bd = torch.as_tensor(b).cuda()
    xa, ia = solve_noalloc(_dev_csr(A), bd, **opts)
    S = Solver(A, spmv_format="csr_vector", **opts)
    xb, ib = S.solve(bd)
    S.close()
    return xa.cpu().numpy(), ia, xb.cpu().numpy(), ib


def _same(xa, ia, xb, ib):
    assert np.array_equal(xa, xb), float(np.max(np.abs(xa - xb)))
    for k in ("status", "iters", "restarts", "rel_resid_true", "rel_resid_recur", "precond_norm"):
        assert ia[k] == ib[k], (k, ia[k], ib[k])


def test_two_calls_in_a_row_match_the_handle_solve():
    # a larger system, then a smaller one: the scratch array keeps the first
    # call's contents, which the second must not depend on
    for A in (poisson3d(48), poisson2d(40)):
        b = rhs_from_solution(A, xstar_uniform(A.n, 1))
        xa, ia, xb, ib = _pair(A, b, tol=1e-10, max_iter=10000)
        _same(xa, ia, xb, ib)
        assert ia["status"] == ppcg.OK and ia["rel_resid_true"] <= 1e-10
        assert ia["iters"] == oracle.pipecg(A, b, tol=1e-10).iters


def test_fixed_iterates_match_handle_and_oracle():
    for A, k in ((random_spd(30000, seed=4), 40), (stencil27_lognormal(16, seed=1), 25)):
        b = rhs_from_solution(A, xstar_uniform(A.n, 1))
        xa, ia, xb, ib = _pair(A, b, fixed_iters=k)
        _same(xa, ia, xb, ib)
        ref = oracle.pipecg(A, b, fixed_iters=k)
        assert ia["iters"] == k
        assert np.linalg.norm(xa - ref.x) / np.linalg.norm(ref.x) <= 1e-10


def test_restart_paths_match_the_handle_solve():
    # tol below the attainable accuracy: restarts, then STAGNATED
    A = stencil27_lognormal(20, seed=2)
    b = rhs_from_solution(A, xstar_uniform(A.n))
    xa, ia, xb, ib = _pair(A, b, tol=1e-18, max_iter=5000, max_restarts=2)
    _same(xa, ia, xb, ib)
    assert ia["status"] == ppcg.STAGNATED and ia["restarts"] == 2


def test_initial_guess_and_largest_size():
    import torch

    A = poisson2d(724)  # 524,176 rows: just below the limit
    assert A.n <= MAX_ROWS
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    x0 = torch.as_tensor(xstar_uniform(A.n, 7) * 0.5).cuda()
    bd = torch.as_tensor(b).cuda()
    xa, ia = solve_noalloc(_dev_csr(A), bd, x0=x0, fixed_iters=30)
    S = Solver(A, spmv_format="csr_vector", fixed_iters=30)
    xb, ib = S.solve(bd, x0=x0)
    S.close()
    _same(xa.cpu().numpy(), ia, xb.cpu().numpy(), ib)
    # x0 may be x itself
    x = x0.clone()
    xc, ic = solve_noalloc(_dev_csr(A), bd, x0=x, out=x, fixed_iters=30)
    assert torch.equal(xc, xa)


def test_rejects_sizes_beyond_the_limit_and_bad_csr():
    import torch

    n = MAX_ROWS + 1
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.arange(n, dtype=torch.int32, device="cuda")
    val = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.full((n,), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ppcg.PPCGError) as e:
        solve_noalloc((rp, ci, val), b, out=x)
    assert e.value.status == ppcg.ERR_INVALID_ARG and "524288" in str(e.value)
    assert bool(torch.all(x == 3.0))
    # a missing diagonal is found on the device
    A = poisson2d(8)
    rp, ci, val = _dev_csr(A)
    val[0] = -1.0
    x = torch.full((A.n,), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ppcg.PPCGError) as e:
        solve_noalloc((rp, ci, val), torch.ones(A.n, dtype=torch.float64, device="cuda"), out=x)
    assert e.value.status == ppcg.ERR_BAD_CSR
    assert bool(torch.all(x == 3.0))
