"""Two host threads use the library at once: creates (with autotuning and
memory releases), graph captures and solves of different systems overlap.
Every result equals a later single-threaded solve of the same system bit for
bit (the autotuner gives every handle of a matrix signature the same layout,
and releases never meet a graph capture in another thread)."""

import threading

import numpy as np
import pytest

from paper_2105_06176_amd.ppcg import Solver
from workloads import poisson3d, random_spd, rhs_from_solution, stencil27_lognormal, xstar_uniform

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_two_threads_create_and_solve_concurrently():
    import torch

    mats = [[poisson3d(36), random_spd(40000, seed=3), stencil27_lognormal(24, seed=1)],
            [random_spd(60000, seed=4), poisson3d(44), stencil27_lognormal(20, seed=2)]]
    bs = [[_dev(rhs_from_solution(A, xstar_uniform(A.n, 7 + k))) for k, A in enumerate(row)] for row in mats]
    # outputs allocated up front: no device allocation inside the threads
    outs = [[torch.empty(A.n, dtype=torch.float64, device="cuda") for A in row] for row in mats]
    torch.cuda.synchronize()
    errors, infos = [], [[None] * len(row) for row in mats]

    def work(t):
        try:
            for k, A in enumerate(mats[t]):
                for _ in range(2):  # each system created, solved and released twice
                    S = Solver(A, tol=1e-10)
                    _, infos[t][k] = S.solve(bs[t][k], out=outs[t][k])
                    S.close()
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(t,)) for t in range(len(mats))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for t, row in enumerate(mats):
        for k, A in enumerate(row):
            assert infos[t][k]["status"] == 0, (t, k, infos[t][k])
            S = Solver(A, tol=1e-10)
            x, info = S.solve(bs[t][k])
            S.close()
            assert np.array_equal(x.cpu().numpy(), outs[t][k].cpu().numpy()), (t, k)
            assert info["iters"] == infos[t][k]["iters"], (t, k)
