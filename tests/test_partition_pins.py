"""Pins of the row-split planner's reference (oracle/partition.py) against
what Section IV-C of the paper and closed forms fix."""

import os

import numpy as np
import pytest

import oracle
from workloads import CSR, poisson3d, random_spd

if os.environ.get("ORACLE_PARTITION"):
    # another copy of oracle/partition.py (the mutation tests plant mistakes in copies)
    import importlib.util

    _spec = importlib.util.spec_from_file_location("partition_under_test", os.environ["ORACLE_PARTITION"])
    P = importlib.util.module_from_spec(_spec)
    _spec.loader.exec_module(P)
else:
    from oracle import partition as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _figure_matrix():
    ents, meta = [], {}
    with open(os.path.join(GOLDEN, "fig_2d_decomposition.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "entry":
                ents.append((int(p[1]) - 1, int(p[2]) - 1, float(p[3])))
            elif p[0] == "nnz1_cpu_entries":
                meta["local"] = [tuple(int(v) - 1 for v in e.split(",")) for e in p[1:]]
            else:
                meta[p[0]] = int(p[1])
    n = meta["n"]
    ents.sort()
    rp = np.zeros(n + 1, np.int32)
    for i, _, _ in ents:
        rp[i + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    A = CSR(n, rp, np.array([e[1] for e in ents], np.int32), np.array([e[2] for e in ents]), "fig")
    return A, meta


def test_figure_example_split_and_local_entries():
    A, meta = _figure_matrix()
    assert A.n == 5 and A.nnz == 15
    # a CPU 1.5x slower than the GPU on the same SpMV: r_cpu = 0.4, nnz_cpu = 6,
    # exactly the non-zeros of the first two rows
    r = P.relative_performance(A.nnz, [1.5, 1.0])
    assert r[0] == pytest.approx(0.4) and r[1] == pytest.approx(0.6)
    b = P.split_rows(A.rp, [1.5, 1.0])
    assert b == [0, meta["N_cpu"], 5]
    nnz1, nnz2, remote = P.decompose(A.rp, A.ci, 0, 2)
    local = [(i, int(A.ci[k])) for i in range(2) for k in range(A.rp[i], A.rp[i + 1]) if int(A.ci[k]) < 2]
    assert sorted(local) == sorted(meta["local"])
    assert nnz1 == 4 and nnz1 + nnz2 == int(A.rp[2])
    assert remote == [2]
    g1, g2, gremote = P.decompose(A.rp, A.ci, 2, 5)
    assert g1 + g2 == A.nnz - int(A.rp[2]) and gremote == [0, 1]


def test_split_takes_equal_or_slightly_fewer_nonzeros():
    A = random_spd(3000, seed=5)
    rng = np.random.default_rng(0)
    for _ in range(20):
        t = rng.uniform(0.1, 5.0, size=2)
        b = P.split_rows(A.rp, t)
        share = A.nnz * P.relative_performance(A.nnz, t)[0]
        assert A.rp[b[1]] <= share
        assert b[1] == A.n or A.rp[b[1] + 1] > share


def test_uniform_rows_closed_form():
    n, L = 1000, 5
    rp = np.arange(n + 1, dtype=np.int64) * L
    for G in (2, 3, 4, 8):
        b = P.split_rows(rp, [1.0] * G)
        assert b == [(n * k) // G for k in range(G)] + [n]


def test_faster_unit_gets_proportionally_more_rows():
    rp = np.arange(10001, dtype=np.int64) * 7
    b = P.split_rows(rp, [3.0, 1.0])  # the second unit is 3x faster
    assert b == [0, 2500, 10000]


def test_slab_halo_of_3d_poisson_is_two_planes():
    s = 12
    A = poisson3d(s)
    plane = s * s
    for z0, z1 in ((0, 4), (4, 8), (3, 12)):
        lo, hi = z0 * plane, z1 * plane
        nnz1, nnz2, remote = P.decompose(A.rp, A.ci, lo, hi)
        faces = (z0 > 0) + (z1 < s)
        assert nnz2 == faces * plane
        assert len(remote) == faces * plane
        assert nnz1 + nnz2 == int(A.rp[hi] - A.rp[lo])
        expect = ([] if z0 == 0 else list(range((z0 - 1) * plane, z0 * plane))) + \
                 ([] if z1 == s else list(range(z1 * plane, (z1 + 1) * plane)))
        assert remote == expect


def test_split_spmv_equals_spmv():
    A = random_spd(800, seed=3)
    x = np.random.default_rng(4).uniform(-1, 1, A.n)
    y = oracle.spmv(A, x)
    # one unit: part 2 is empty, the sum is the CSR-order sum exactly
    assert np.array_equal(P.split_spmv(A.rp, A.ci, A.val, x, 0, A.n), y)
    for lo, hi in ((0, 300), (300, 800), (123, 456)):
        ys = P.split_spmv(A.rp, A.ci, A.val, x, lo, hi)
        rowabs = np.abs(A.to_scipy()) @ np.abs(x)
        assert np.all(np.abs(ys - y[lo:hi]) <= 4 * np.finfo(float).eps * rowabs[lo:hi])


def test_figure_matrix_other_splits_by_hand():
    """Counted by hand from the figure pattern (1-based rows 1-3 hold columns
    1-3, and row 3 also column 4)."""
    A, _ = _figure_matrix()
    assert P.decompose(A.rp, A.ci, 0, 3) == (9, 1, [3])
    assert P.decompose(A.rp, A.ci, 3, 5) == (4, 1, [2])
    assert P.decompose(A.rp, A.ci, 0, 5) == (15, 0, [])


# ---------------------------------------------------------------- the library's planner (host only)

def test_library_split_rows_matches_reference():
    from paper_2105_06176_amd import ppcg

    rng = np.random.default_rng(7)
    mats = [random_spd(2000, seed=1), poisson3d(10), _figure_matrix()[0]]
    for A in mats:
        for parts in (1, 2, 3, 5, 8):
            for _ in range(6):
                t = rng.uniform(0.05, 3.0, size=parts)
                assert ppcg.split_rows(A.rp, t) == P.split_rows(A.rp, t), (A.name, parts, t)
    A, meta = _figure_matrix()
    assert ppcg.split_rows(A.rp, [1.5, 1.0]) == [0, meta["N_cpu"], 5]


def test_library_split_rows_rejects_bad_input():
    from paper_2105_06176_amd import ppcg

    rp = np.array([0, 2, 4], np.int32)
    with pytest.raises(ppcg.PPCGError):
        ppcg.split_rows(rp, [1.0, 0.0])
    with pytest.raises(ppcg.PPCGError):
        ppcg.split_rows(rp, [1.0, float("nan")])
    with pytest.raises(ppcg.PPCGError):
        ppcg.split_rows(np.array([0, 3, 2], np.int32), [1.0, 1.0])
    # no non-zeros: the first unit takes every row
    assert ppcg.split_rows(np.zeros(4, np.int32), [1.0, 2.0]) == [0, 3, 3]
