"""Batched solves that reuse the engine kept on the batch's first handle.

ppcg_solve_batch keeps its engine (buffers, streams, captured graphs) and
its staging table on the first handle and reuses them for the next batch
that handle leads, with at most as many systems.  Each batch must give the
results of a fresh one: bitwise equal to the solo solves, whatever batches
ran before on the same engine (another composition, fixed iterations, an
initial guess, host vectors, a larger batch that replaces the engine).
"""

import numpy as np
import pytest

import oracle
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Solver, solve_batch
from workloads import poisson2d, poisson3d, random_spd, rhs_from_solution, shifted, stencil27_lognormal, xstar_uniform

pytestmark = pytest.mark.gpu


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _systems():
    # two-launch or single-launch (autotuned), one-workgroup, sorted rows
    return [poisson2d(100), poisson3d(30), stencil27_lognormal(16, seed=1), random_spd(9000, seed=2),
            shifted(poisson2d(40), 0.05)]


def test_batches_on_one_engine_equal_fresh_solves():
    mats = _systems()
    bs = [rhs_from_solution(A, xstar_uniform(A.n, 70 + i)) for i, A in enumerate(mats)]
    solo = [host(Solver(A, tol=1e-10).solve(dev(b))[0]) for A, b in zip(mats, bs)]
    S = [Solver(A, tol=1e-10) for A in mats]
    bd = [dev(b) for b in bs]

    def full_batch(tag):
        xs, infos = solve_batch(S, bd)
        for i, (x, info) in enumerate(zip(xs, infos)):
            assert info["status"] == ppcg.OK, (tag, i, info)
            assert np.array_equal(host(x), solo[i]), (tag, mats[i].name)

    full_batch("first")
    full_batch("repeat")
    # a smaller batch of other composition led by the same handle: fixed
    # iterations, one system with an initial guess
    S[0].set_options(fixed_iters=25)
    S[3].set_options(fixed_iters=25)
    g = xstar_uniform(mats[3].n, 9) * 0.5
    xs, infos = solve_batch([S[0], S[3]], [bd[0], bd[3]], x0s=[None, dev(g)])
    assert [i["iters"] for i in infos] == [25, 25]
    assert relerr(host(xs[0]), oracle.pipecg(mats[0], bs[0], fixed_iters=25).x) <= 1e-10
    assert relerr(host(xs[1]), oracle.pipecg(mats[3], bs[3], x0=g, fixed_iters=25).x) <= 1e-10
    S[0].set_options(fixed_iters=0, tol=1e-10)
    S[3].set_options(fixed_iters=0, tol=1e-10)
    full_batch("after a smaller one")
    for s in S:
        s.close()


def test_larger_batch_with_host_vectors_replaces_the_engine():
    import torch

    mats = _systems()
    bs = [rhs_from_solution(A, xstar_uniform(A.n, 90 + i)) for i, A in enumerate(mats)]
    S = [Solver(A, tol=1e-10) for A in mats[:3]]
    xs, _ = solve_batch(S, [dev(b) for b in bs[:3]])
    first = [host(x) for x in xs]
    # the same first handle leads a larger batch; two systems keep their
    # vectors in host memory
    Sh = [Solver(A, tol=1e-10, vec_mem="host") for A in mats[3:]]
    allS = S + Sh
    ins = [dev(b) for b in bs[:3]] + [torch.as_tensor(b) for b in bs[3:]]
    outs = [s._alloc() for s in S] + [torch.zeros(A.n, dtype=torch.float64) for A in mats[3:]]
    xs, infos = solve_batch(allS, ins, outs=outs)
    for i, (x, info) in enumerate(zip(xs, infos)):
        assert info["status"] == ppcg.OK, (i, info)
        xh = host(x)
        assert oracle.true_relres(mats[i], bs[i], xh) <= 1e-10
        if i < 3:
            assert np.array_equal(xh, first[i])
        else:
            ref = torch.zeros(mats[i].n, dtype=torch.float64)
            allS[i].solve(torch.as_tensor(bs[i]), out=ref)
            assert np.array_equal(xh, ref.numpy())
    for s in allS:
        s.close()
