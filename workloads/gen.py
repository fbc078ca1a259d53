"""Seeded generators for the synthetic SPD workloads.

Every matrix is returned in CSR form with int32 row pointers and column
indices and float64 values; columns inside a row are strictly ascending and
every row stores its diagonal.  Grid points are numbered lexicographically
with x varying fastest.  Dirichlet neighbours outside the grid are simply
absent from a row.

Workloads (the paper's experiment protocol and the benchmark shapes):

* ``poisson2d(n)``  - 5-point Laplacian, diagonal 4, off-diagonals -1.
* ``poisson3d(n)``  - 7-point Laplacian, diagonal 6, off-diagonals -1.
* ``poisson125(n)`` - 125-point box stencil (the paper's large Poisson
  matrices, Section VI-B, Table 2), diagonal 124, off-diagonals -1.
* ``stencil27_lognormal(n, seed, shift)`` - 27-point box stencil whose
  off-diagonal entries are ``-k`` with one ``k = exp(Z)``, ``Z ~ N(0,1)``, per
  undirected edge; the diagonal is the row's absolute off-diagonal sum plus
  ``shift``.
* ``random_spd(n, seed)`` - symmetric sparse matrix with 8 uniformly drawn
  off-diagonal columns per row, mirrored, values uniform in [-1, 0),
  duplicates summed; diagonal = absolute row sum + 1e-2.
* ``batch_c4(seed, count)`` - sizes and shifts of the 256-system batch of
  shifted 2-D Poisson problems.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class CSR:
    """Square sparse matrix in compressed sparse row form."""

    n: int
    rp: np.ndarray  # int32[n+1]
    ci: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.ci, self.rp), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def diag(self) -> np.ndarray:
        return self.to_scipy().diagonal()


def _coords(dims: Sequence[int]) -> List[np.ndarray]:
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    out = []
    stride = 1
    for d in dims:
        out.append((idx // stride) % d)
        stride *= d
    return out


def _box_offsets(ndim: int, radius: int) -> List[Tuple[int, ...]]:
    rng = range(-radius, radius + 1)
    if ndim == 2:
        offs = [(dx, dy) for dy in rng for dx in rng]
    else:
        offs = [(dx, dy, dz) for dz in rng for dy in rng for dx in rng]
    return offs


def _linear(off: Tuple[int, ...], dims: Sequence[int]) -> int:
    lin, stride = 0, 1
    for o, d in zip(off, dims):
        lin += o * stride
        stride *= d
    return lin


def _stencil_pattern(dims: Sequence[int], offsets: Sequence[Tuple[int, ...]]):
    """Column table (n, K) with -1 where the neighbour lies outside the grid.

    ``offsets`` are sorted by linear offset so every row's columns ascend.
    """
    offsets = sorted(offsets, key=lambda o: _linear(o, dims))
    coords = _coords(dims)
    n = int(np.prod(dims))
    cols = np.empty((n, len(offsets)), dtype=np.int32)
    idx = np.arange(n, dtype=np.int64)
    for k, off in enumerate(offsets):
        ok = np.ones(n, dtype=bool)
        for c, o, d in zip(coords, off, dims):
            if o:
                ok &= (c + o >= 0) & (c + o < d)
        lin = _linear(off, dims)
        cols[:, k] = np.where(ok, idx + lin, -1)
    return cols, offsets


def _compress(cols: np.ndarray, vals: np.ndarray, name: str) -> CSR:
    valid = cols >= 0
    lens = valid.sum(axis=1)
    n = cols.shape[0]
    nnz = int(lens.sum())
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    return CSR(n, rp.astype(np.int32), cols[valid].astype(np.int32), vals[valid].astype(np.float64), name)


def _constant_stencil(dims, radius_or_offsets, diag: float, off: float, name: str) -> CSR:
    cols, offsets = _stencil_pattern(dims, radius_or_offsets)
    vals = np.full(cols.shape, off, dtype=np.float64)
    zero = [k for k, o in enumerate(offsets) if not any(o)][0]
    vals[:, zero] = diag
    return _compress(cols, vals, name)


def poisson2d(n: int) -> CSR:
    """2-D 5-point Dirichlet Laplacian on an n x n grid (N = n^2)."""
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    return _constant_stencil((n, n), offs, 4.0, -1.0, f"poisson2d_{n}")


def poisson3d(n: int) -> CSR:
    """3-D 7-point Dirichlet Laplacian on an n^3 grid (N = n^3)."""
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    return _constant_stencil((n, n, n), offs, 6.0, -1.0, f"poisson3d_{n}")


def poisson125(n: int) -> CSR:
    """125-point (5x5x5 box) Poisson-type matrix on an n^3 grid.

    The paper gives only the stencil width and the sizes (Table 2); the
    values are taken as diagonal 124 and off-diagonal -1, which is weakly
    diagonally dominant and irreducible, hence SPD.
    """
    return _constant_stencil((n, n, n), _box_offsets(3, 2), 124.0, -1.0, f"poisson125_{n}")


def stencil27_lognormal(n: int, seed: int = 0, shift: float = 1e-3) -> CSR:
    """27-point variable-coefficient stencil, lognormal edge weights.

    One weight per undirected edge: for each of the 13 neighbour directions
    with positive linear offset ``d`` an array ``K_d`` of ``n^3`` draws
    ``exp(N(0,1))`` is taken from ``default_rng(seed)`` (directions in
    ascending linear offset).  Edge ``{i, i+d}`` has weight ``K_d[i]`` and
    both ``a[i, i+d]`` and ``a[i+d, i]`` equal ``-K_d[i]``.  The diagonal is the
    row's absolute off-diagonal sum plus ``shift``, so ``A = L + shift*I``
    with ``L`` a weighted graph Laplacian.
    """
    dims = (n, n, n)
    cols, offsets = _stencil_pattern(dims, _box_offsets(3, 1))
    N = n ** 3
    lin = [_linear(o, dims) for o in offsets]
    rng = np.random.default_rng(seed)
    weights = {}
    for d in sorted(l for l in lin if l > 0):
        weights[d] = np.exp(rng.standard_normal(N))
    vals = np.zeros(cols.shape, dtype=np.float64)
    idx = np.arange(N, dtype=np.int64)
    zero = lin.index(0)
    for k, d in enumerate(lin):
        if d == 0:
            continue
        valid = cols[:, k] >= 0
        if d > 0:
            w = weights[d]
            vals[:, k] = np.where(valid, -w, 0.0)
        else:
            w = weights[-d]
            src = np.where(valid, idx + d, 0)
            vals[:, k] = np.where(valid, -w[src], 0.0)
    vals[:, zero] = np.abs(vals).sum(axis=1) + shift
    return _compress(cols, vals, f"stencil27_lognormal_{n}")


def random_spd(n: int, seed: int = 0, draws: int = 8, dominance: float = 1e-2) -> CSR:
    """Random symmetric sparse SPD matrix (about 16 off-diagonals per row).

    Each row draws ``draws`` columns uniformly from the other ``n-1`` indices
    with values uniform in [-1, 0); draws that land on the same unordered
    pair are summed and the result is mirrored, and the diagonal is the absolute off-diagonal row sum plus
    ``dominance`` (strict diagonal dominance, so SPD).
    """
    import scipy.sparse as sp

    if n < 2:
        raise ValueError("random_spd needs n >= 2")
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), draws)
    cols = rng.integers(0, n - 1, size=n * draws, dtype=np.int64)
    cols = cols + (cols >= rows)  # skip the diagonal
    vals = rng.uniform(-1.0, 0.0, size=n * draws)
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    upper = sp.coo_matrix((vals, (lo, hi)), shape=(n, n)).tocsr()
    upper.sum_duplicates()
    off = (upper + upper.T).tocsr()  # exact mirror of the summed upper triangle
    off.sort_indices()
    d = np.asarray(abs(off).sum(axis=1)).ravel() + dominance
    A = (off + sp.diags(d)).tocsr()
    A.sort_indices()
    return CSR(n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64),
               f"random_spd_{n}_{seed}")


def shifted(A: CSR, sigma: float) -> CSR:
    """Return A + sigma*I (A must store its diagonal)."""
    val = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    on_diag = A.ci == rows
    val[on_diag] += sigma
    return CSR(A.n, A.rp.copy(), A.ci.copy(), val, f"{A.name}+{sigma:g}I")


def xstar_uniform(n: int, seed: int = 1) -> np.ndarray:
    """Exact solution with entries uniform in [-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def xstar_paper(n: int) -> np.ndarray:
    """The paper's exact solution: every entry 1/sqrt(N) (Section VI)."""
    return np.full(n, 1.0 / math.sqrt(n))


def rhs_from_solution(A: CSR, xstar: np.ndarray) -> np.ndarray:
    """b = A x* in float64 (a library sparse product, input preparation only)."""
    return np.asarray(A.to_scipy() @ xstar, dtype=np.float64)


def poisson2d_eigpair(n: int, j: int, k: int):
    """Closed-form eigenpair (lambda, v) of the 2-D Dirichlet 5-point Laplacian."""
    t = np.arange(1, n + 1)
    vx = np.sin(j * np.pi * t / (n + 1))
    vy = np.sin(k * np.pi * t / (n + 1))
    v = np.outer(vy, vx).ravel()  # x fastest
    lam = 4 * math.sin(j * math.pi / (2 * (n + 1))) ** 2 + 4 * math.sin(k * math.pi / (2 * (n + 1))) ** 2
    return lam, v


def poisson3d_eigpair(n: int, j: int, k: int, l: int):
    """Closed-form eigenpair (lambda, v) of the 3-D Dirichlet 7-point Laplacian."""
    t = np.arange(1, n + 1)
    vx = np.sin(j * np.pi * t / (n + 1))
    vy = np.sin(k * np.pi * t / (n + 1))
    vz = np.sin(l * np.pi * t / (n + 1))
    v = (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).ravel()
    lam = sum(4 * math.sin(a * math.pi / (2 * (n + 1))) ** 2 for a in (j, k, l))
    return lam, v


def nnz_poisson2d(n: int) -> int:
    return 5 * n * n - 4 * n


def nnz_poisson3d(n: int) -> int:
    return 7 * n ** 3 - 6 * n ** 2


def nnz_stencil27(n: int) -> int:
    return (3 * n - 2) ** 3


def nnz_poisson125(n: int) -> int:
    return (5 * n - 6) ** 3


def batch_c4(seed: int = 0, count: int = 256, side_lo: int = 32, side_hi: int = 512):
    """(side, shift) of each system of the shifted 2-D Poisson batch.

    Sides are integers uniform in [side_lo, side_hi] and shifts uniform in
    [0, 0.5), both from ``default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    shifts = rng.uniform(0.0, 0.5, size=count)
    return [(int(s), float(h)) for s, h in zip(sides, shifts)]
