"""Parity at the workloads' full sizes, in the configurations bench.py times:
the 27-point lognormal stencil at 160^3 (FP64 and FP32 values), the 256-system
batch, Table 2's 125-point Poisson matrix at side 165, and the 4.1M-row random
sparse SPD matrix.  Reference values
the oracle cannot afford at this size inline come from tests/golden (written by
make_c3_p125_reference.py from the oracle only); the rest is checked through
properties that hold at any size (true residual recomputed by the oracle,
SpMV bit for bit)."""

import os

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Solver, solve_batch
from workloads import (batch_c4, poisson125, poisson2d, random_spd, rhs_from_solution, shifted,
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


def _golden(name, key):
    vals, meta = {}, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == key:
                vals[int(p[1])] = float(p[2])
            else:
                meta[p[0]] = float(p[1])
    return vals, meta


def _golden_all(name):
    """Every sampled vector of a golden file ({key: {index: value}}) and its
    scalar entries."""
    vecs, meta = {}, {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if len(p) == 3:
                vecs.setdefault(p[0], {})[int(p[1])] = float(p[2])
            else:
                meta[p[0]] = float(p[1])
    return vecs, meta


def _check_sampled(x, vals, meta, k):
    idx = np.array(sorted(vals))
    assert relerr(x[idx], np.array([vals[i] for i in idx])) <= 1e-10
    assert abs(np.linalg.norm(x) - meta[f"norm_x{k}"]) <= 1e-10 * meta[f"norm_x{k}"]


def test_c3_stencil27_160_full_size():
    A = stencil27_lognormal(160, seed=0, shift=1e-3)
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    vals, meta = _golden("c3_stencil27_160.txt", "x10")
    assert (meta["n"], meta["nnz"]) == (A.n, A.nnz)
    S = Solver(A, fixed_iters=10, spmv_format="sell")
    xt = xstar_uniform(A.n, 5)
    assert np.array_equal(host(S.spmv(dev(xt))), oracle.spmv(A, xt))
    x, info = S.solve(dev(b))
    assert info["iters"] == 10
    _check_sampled(host(x), vals, meta, 10)
    # x_200: far enough in that the rounding order of the dot products moves
    # the iterate; the oracle's two roundings bound how far
    g, gm = _golden_all("c3_stencil27_160_x200.txt")
    idx = np.array(sorted(g["x200"]))
    xa = np.array([g["x200"][i] for i in idx])
    xc = np.array([g["x200c"][i] for i in idx])
    sens = max(relerr(xc, xa), abs(gm["norm_x200c"] - gm["norm_x200"]) / gm["norm_x200"])
    S.set_options(fixed_iters=200, spmv_format="sell")
    x, info = S.solve(dev(b))
    assert info["iters"] == 200
    x = host(x)
    e = max(relerr(x[idx], xa), abs(np.linalg.norm(x) - gm["norm_x200"]) / gm["norm_x200"])
    print(f"C3 x_200: gpu vs oracle {e:.2e}, oracle rounding sensitivity {sens:.2e}")
    assert e <= max(1e-10, 10 * sens)
    # to 1e-10 in FP64 and both mixed precisions: true residuals recomputed by
    # the oracle, and the distance to the oracle's own solution.  A = L + 1e-3 I
    # with L a graph Laplacian (positive semidefinite), so ||A^-1||_2 <= 1e3 and
    # two solutions with residuals r1, r2 differ by at most 1e3 (||r1|| + ||r2||)
    # in the 2-norm, hence in every entry.
    t, tm = _golden_all("c3_stencil27_160_tol.txt")
    ti = np.array(sorted(t["x_tol"]))
    xo = np.array([t["x_tol"][i] for i in ti])
    iters = {}
    for prec in ("fp64", "mixed_values", "mixed"):
        S.set_options(tol=1e-10, max_iter=20000, spmv_format="sell", precision=prec)
        xp, ip = S.solve(dev(b))
        xp = host(xp)
        rel = oracle.true_relres(A, b, xp)
        assert ip["status"] == ppcg.OK and rel <= 1e-10, (prec, ip)
        bound = 1e3 * (rel + tm["rel_true"]) * tm["bnorm"]
        diff = float(np.max(np.abs(xp[ti] - xo)))
        print(f"C3 {prec}: {ip['iters']} iterations (oracle {int(tm['iters'])}), true residual {rel:.2e}, "
              f"sampled rel. diff vs oracle solution {relerr(xp[ti], xo):.2e}, max |diff| {diff:.2e} "
              f"(bound {bound:.2e})")
        assert diff <= bound
        iters[prec] = ip["iters"]
    assert abs(iters["fp64"] - tm["iters"]) <= 0.05 * tm["iters"]
    assert iters["mixed_values"] <= 1.15 * iters["fp64"] + 5


def test_c4_full_batch():
    spec = batch_c4(seed=0, count=256)
    mats = [shifted(poisson2d(side), sh) for side, sh in spec]
    bs = [rhs_from_solution(A, xstar_uniform(A.n, 1000 + i)) for i, A in enumerate(mats)]
    solvers = [Solver(A, tol=1e-10, spmv_format="sell") for A in mats]
    xs, infos = solve_batch(solvers, [dev(b) for b in bs])
    for A, b, x, info in zip(mats, bs, xs, infos):
        assert info["status"] == ppcg.OK
        assert oracle.true_relres(A, b, host(x)) <= 1e-10
    # iteration counts against the oracle on a sample of systems of every size class
    order = np.argsort([A.n for A in mats])
    for k in list(order[:3]) + list(order[len(order) // 2: len(order) // 2 + 2]):
        ref = oracle.pipecg(mats[k], bs[k], tol=1e-10)
        assert abs(infos[k]["iters"] - ref.iters) <= 2, (mats[k].n, infos[k]["iters"], ref.iters)
    for S in solvers:
        S.close()


@pytest.fixture(scope="module")
def p125():
    A = poisson125(165)
    return A, rhs_from_solution(A, xstar_paper(A.n))


@pytest.mark.parametrize("vflag", [ppcg.FLAG_SELL_VALUE_TABLE, ppcg.FLAG_SELL_FULL_VALUES,
                                   ppcg.FLAG_SELL_VALUE_TABLE | ppcg.FLAG_SELL_SHARED_OFFSETS,
                                   ppcg.FLAG_SELL_VALUE_TABLE | ppcg.FLAG_SELL_NO_SHARED_OFFSETS])
def test_table2_125pt_side165_full_size(p125, vflag):
    """Table 2's matrix at full size with its three distinct values read
    through the one-byte table (as the autotuner picks it) and as 8-byte
    values, on the chunks' shared offset lists and on per-entry columns: the
    SpMV equals the oracle's bit for bit, and x_5 and the iteration count
    under the paper's protocol match the stored values."""
    A, b = p125
    vals, meta = _golden("p125_side165.txt", "x5")
    assert (meta["n"], meta["nnz"]) == (A.n, A.nnz)
    S = Solver(A, fixed_iters=5, flags=vflag)
    mi = S.matrix_info()
    assert mi["value_bytes"] == (1 if vflag & ppcg.FLAG_SELL_VALUE_TABLE else 8)
    if vflag & ppcg.FLAG_SELL_SHARED_OFFSETS:
        assert mi["col_index_bytes"] == 0
    if vflag & ppcg.FLAG_SELL_NO_SHARED_OFFSETS:
        assert mi["col_index_bytes"] in (2, 4)
    xs = xstar_uniform(A.n, 5)
    assert np.array_equal(host(S.spmv(dev(xs))), oracle.spmv(A, xs))
    x, info = S.solve(dev(b))
    assert info["iters"] == 5
    _check_sampled(host(x), vals, meta, 5)
    S.set_options(tol=1e-5, stop="abs", max_iter=10000)
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK
    assert abs(info["iters"] - int(meta["abs1e-5_iters"])) <= 2
    assert info["precond_norm"] < 1e-5
    S.close()


def test_random_spd_4_1m_full_size():
    """The random sparse SPD matrix of the throughput measurements at full
    size (4,096,000 rows, about 17 entries per row, uniform random columns)
    in the autotuned storage: the SpMV equals the oracle's bit for bit, 10
    fixed iterates meet the 1e-10 bar against the oracle's, and the solve to
    1e-10 meets it (true residual recomputed by the oracle)."""
    A = random_spd(4_096_000, seed=0)
    b = rhs_from_solution(A, xstar_uniform(A.n, 1))
    S = Solver(A, fixed_iters=10)
    xs = xstar_uniform(A.n, 5)
    assert np.array_equal(host(S.spmv(dev(xs))), oracle.spmv(A, xs))
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK and info["iters"] == 10, info
    assert relerr(host(x), oracle.pipecg(A, b, fixed_iters=10).x) <= 1e-10
    S.set_options(fixed_iters=0, tol=1e-10)
    x, info = S.solve(dev(b))
    assert info["status"] == ppcg.OK, info
    assert oracle.true_relres(A, b, host(x)) <= 1e-10
    S.close()
