"""GPU parity of one unit's share of A under the 2-D decomposition (Section
IV-C): the two-part SpMV against the oracle's definition (part 1 over the
local-column entries, part 2 over the others, each summed in stored order,
then added) bit for bit, and the halo bookkeeping against the oracle's
decomposition."""

import numpy as np
import pytest

from oracle import partition as P
from paper_2105_06176_amd import ppcg
from paper_2105_06176_amd.ppcg import Shard
from workloads import poisson2d, poisson3d, random_spd, stencil27_lognormal, xstar_uniform

pytestmark = pytest.mark.gpu


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _check_shard(A, lo, hi, seed=3):
    import torch

    x = xstar_uniform(A.n, seed)
    S = Shard(A, lo, hi)
    info = S.info()
    nnz1, nnz2, remote = P.decompose(A.rp, A.ci, lo, hi)
    assert (info["nnz_local"], info["nnz_remote"], info["halo"]) == (nnz1, nnz2, len(remote))
    assert list(S.halo_columns()) == remote
    xg = dev(x)
    xh = torch.empty(max(len(remote), 1), dtype=torch.float64, device="cuda")
    S.gather(xg, xh)
    assert np.array_equal(xh.cpu().numpy()[:len(remote)], x[remote])
    y = torch.empty(hi - lo, dtype=torch.float64, device="cuda")
    S.spmv(dev(x[lo:hi]), xh, y, parts=3)
    ref = P.split_spmv(A.rp, A.ci, A.val, x, lo, hi)
    assert np.array_equal(y.cpu().numpy(), ref), (A.name, lo, hi)
    # part 1 alone, then part 2 on top: the same result
    y2 = torch.empty_like(y)
    S.spmv(dev(x[lo:hi]), xh, y2, parts=1)
    S.spmv(dev(x[lo:hi]), xh, y2, parts=2)
    assert np.array_equal(y2.cpu().numpy(), ref)
    S.close()
    return info


@pytest.mark.parametrize("gen", [lambda: random_spd(3001, seed=2), lambda: poisson3d(20),
                                 lambda: stencil27_lognormal(12, seed=3), lambda: poisson2d(37)])
def test_shards_of_a_split_match_oracle(gen):
    A = gen()
    rng = np.random.default_rng(11)
    for parts in (1, 2, 3, 8):
        t = rng.uniform(0.5, 2.0, size=parts)
        b = ppcg.split_rows(A.rp, t)
        assert b == P.split_rows(A.rp, t)
        for k in range(parts):
            if b[k + 1] > b[k]:
                _check_shard(A, b[k], b[k + 1])


def test_single_row_and_ragged_shards():
    A = random_spd(500, seed=9)
    for lo, hi in ((0, 1), (499, 500), (17, 83), (64, 128), (1, 499)):
        _check_shard(A, lo, hi)


def test_shard_rejects_bad_ranges():
    A = poisson2d(8)
    for lo, hi in ((-1, 5), (5, 5), (3, 65)):
        with pytest.raises(ppcg.PPCGError):
            Shard(A, lo, hi)


def test_full_size_slabs_of_128_cube():
    """3-D 7-point 128^3: a slab of 16 whole planes has exactly two halo
    planes; the performance-model slab (equal speeds, 8 units) cuts planes at
    non-zero counts, so its halo is two planes plus a few rows; both two-part
    SpMVs equal the oracle's on the whole slab."""
    A = poisson3d(128)
    plane = 128 * 128
    info = _check_shard(A, 3 * 16 * plane, 4 * 16 * plane)
    assert info["halo"] == info["nnz_remote"] == 2 * plane
    assert info["boundary_rows"] == 2 * plane
    b = ppcg.split_rows(A.rp, [1.0] * 8)
    info = _check_shard(A, b[3], b[4])
    assert 2 * plane <= info["halo"] <= 2 * plane + 2 * 128


def test_shard_timing():
    import torch

    A = poisson3d(64)
    b = ppcg.split_rows(A.rp, [1.0] * 4)
    S = Shard(A, b[1], b[2])
    h = S.info()["halo"]
    xg = dev(xstar_uniform(A.n, 1))
    ms1, msg, ms2 = S.time(xg, xg[b[1]:b[2]].contiguous(), torch.empty(h, dtype=torch.float64, device="cuda"),
                           torch.empty(b[2] - b[1], dtype=torch.float64, device="cuda"), iters=10)
    assert ms1 > 0 and msg > 0 and ms2 > 0
