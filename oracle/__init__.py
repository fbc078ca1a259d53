"""CPU FP64 oracle for the Pipelined PCG solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it,
and it shares no code with the HIP path: the arithmetic lives in
``ppcg_oracle.c`` (plain sequential C, FP64, no FMA contraction); this module
only marshals numpy arrays through ctypes.

Functions and the passages they follow (Tiwari & Vadhiyar, arXiv 2105.06176):

* ``spmv``      - sparse matrix-vector product with A in CSR (Section V-A).
* ``jacobi``    - inverse diagonal of A, the Jacobi preconditioner (Section V-A).
* ``dot``       - FP64 dot product, summed left to right, or with Neumaier's
                  compensated summation (``dots="comp"``; every solver takes
                  the same switch for all of its dot products).
* ``pcg``       - Algorithm 1, PCG (Section III-A).
* ``pipecg``    - Algorithm 2, PIPECG (Section III-B).
* ``true_relres`` - ||b - A x|| / ||b||.

Parity pins (tests/test_oracle_pins.py) tie these to facts fixed outside the
oracle: dense Cholesky and exact rational solutions, the Galerkin
characterisation of the CG iterates, closed-form Poisson eigenpairs, finite
termination, and the agreement of Algorithms 1 and 2.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PPCG_ORACLE_LIB selects another build of the oracle (the tests' sanitized build)
_LIB_PATH = os.environ.get("PPCG_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
_lib = None

OK, NOT_CONVERGED, BREAKDOWN, STAGNATED, BAD_INPUT = 0, 1, 2, 3, -1
STOP_REL, STOP_ABS = 0, 1


class _Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("status", ctypes.c_int),
        ("pad", ctypes.c_int),
        ("rel_true", ctypes.c_double),
        ("rel_recur", ctypes.c_double),
        ("precond_norm", ctypes.c_double),
        ("bnorm", ctypes.c_double),
    ]


@dataclasses.dataclass
class Result:
    x: np.ndarray
    iters: int
    restarts: int
    status: int
    rel_true: float
    rel_recur: float
    precond_norm: float
    bnorm: float
    hist: Optional[np.ndarray] = None
    state: Optional[dict] = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ORACLE_LIB names another build of ppcg_oracle.c; the mutation tests use
    # it to load copies with a planted mistake in place of the oracle.
    path = os.environ.get("ORACLE_LIB", _LIB_PATH)
    if path == _LIB_PATH and (not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
            os.path.join(HERE, "ppcg_oracle.c"))):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    lib.ora_spmv.argtypes = [I, P, P, P, P, P]
    lib.ora_spmv.restype = None
    lib.ora_dot.argtypes = [I, P, P]
    lib.ora_dot.restype = D
    lib.ora_set_dot_mode.argtypes = [I]
    lib.ora_set_dot_mode.restype = None
    lib.ora_jacobi.argtypes = [I, P, P, P, P]
    lib.ora_jacobi.restype = I
    lib.ora_true_relres.argtypes = [I, P, P, P, P, P]
    lib.ora_true_relres.restype = D
    lib.ora_pcg.argtypes = [I, P, P, P, P, P, P, D, I, I, I, I, ctypes.POINTER(_Info), P, I]
    lib.ora_pcg.restype = I
    lib.ora_pipecg.argtypes = [I, P, P, P, P, P, P, D, I, I, I, I, ctypes.POINTER(_Info), P, I, P]
    lib.ora_pipecg.restype = I
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _csr(A):
    rp = np.ascontiguousarray(A.rp, dtype=np.int32)
    ci = np.ascontiguousarray(A.ci, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, val


def spmv(A, x: np.ndarray) -> np.ndarray:
    lib = _load()
    rp, ci, val = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n, dtype=np.float64)
    lib.ora_spmv(A.n, _p(rp), _p(ci), _p(val), _p(x), _p(y))
    return y


_DOT_MODES = {"seq": 0, "comp": 1}


def dot(a: np.ndarray, b: np.ndarray, dots: str = "seq") -> float:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    lib.ora_set_dot_mode(_DOT_MODES[dots])
    try:
        return lib.ora_dot(a.size, _p(a), _p(b))
    finally:
        lib.ora_set_dot_mode(0)


def jacobi(A) -> np.ndarray:
    lib = _load()
    rp, ci, val = _csr(A)
    d = np.empty(A.n, dtype=np.float64)
    if lib.ora_jacobi(A.n, _p(rp), _p(ci), _p(val), _p(d)) != 0:
        raise ValueError("matrix has a missing or non-positive diagonal")
    return d


def true_relres(A, b: np.ndarray, x: np.ndarray) -> float:
    lib = _load()
    rp, ci, val = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.ora_true_relres(A.n, _p(rp), _p(ci), _p(val), _p(b), _p(x))


_STATE_NAMES = ("x", "r", "u", "w", "m", "n", "z", "q", "s", "p")
_SCALAR_NAMES = ("gamma", "delta", "uu", "rr", "alpha_prev", "gamma_prev", "beta_prev")


def _run(which: str, A, b, x0=None, tol=1e-8, maxit=10000, fixed_iters=0, stop=STOP_REL,
         max_restarts=3, history=False, state=False, dots="seq") -> Result:
    lib = _load()
    mode = _DOT_MODES[dots]
    rp, ci, val = _csr(A)
    n = A.n
    b = np.ascontiguousarray(b, dtype=np.float64)
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    x = np.empty(n, dtype=np.float64)
    info = _Info()
    hist_len = (fixed_iters if fixed_iters > 0 else maxit) + 1 if history else 0
    hist = np.full(hist_len, np.nan) if history else None
    st = np.zeros(10 * n + 7) if state else None
    args = [n, _p(rp), _p(ci), _p(val), _p(b), _p(x0a), _p(x), float(tol), int(maxit), int(fixed_iters),
            int(stop), int(max_restarts), ctypes.byref(info), _p(hist), hist_len]
    lib.ora_set_dot_mode(mode)
    try:
        if which == "pcg":
            lib.ora_pcg(*args)
        else:
            lib.ora_pipecg(*args, _p(st))
    finally:
        lib.ora_set_dot_mode(0)
    res = Result(x, info.iters, info.restarts, info.status, info.rel_true, info.rel_recur,
                 info.precond_norm, info.bnorm)
    if history:
        res.hist = hist[: min(info.iters + 1, hist_len)]
    if state:
        d = {k: st[i * n:(i + 1) * n].copy() for i, k in enumerate(_STATE_NAMES)}
        for j, k in enumerate(_SCALAR_NAMES):
            d[k] = float(st[10 * n + j])
        res.state = d
    return res


def pcg(A, b, **kw) -> Result:
    """Algorithm 1 (PCG) with the Jacobi preconditioner, FP64."""
    kw.pop("state", None)
    return _run("pcg", A, b, **kw)


def pipecg(A, b, **kw) -> Result:
    """Algorithm 2 (PIPECG) with the Jacobi preconditioner, FP64."""
    return _run("pipecg", A, b, **kw)


# ---------------------------------------------------------------- PIPECG-OpenMP
# The paper's CPU baseline (Sections V-A and V-B): Algorithm 2 on host threads
# with the vector-update loops merged.  A timing build, not the checker: its
# reductions are summed per thread, so it agrees with ``pipecg`` to rounding.
_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")
_omp = None


def _load_omp():
    global _omp
    if _omp is None:
        if not os.path.exists(_OMP_PATH):
            raise RuntimeError(f"{_OMP_PATH} is missing: run oracle/build.py")
        L = ctypes.CDLL(_OMP_PATH)
        P = ctypes.c_void_p
        L.omp_pipecg.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.omp_pipecg.restype = ctypes.c_int
        L.omp_default_threads.argtypes = []
        L.omp_default_threads.restype = ctypes.c_int
        _omp = L
    return _omp


def omp_default_threads() -> int:
    return int(_load_omp().omp_default_threads())


def pipecg_openmp(A, b, x0=None, tol=1e-8, maxit=10000, fixed_iters=0, stop=STOP_REL, threads=None):
    """PIPECG-OpenMP: returns (x, status, iterations)."""
    L = _load_omp()
    rp, ci, val = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    it = ctypes.c_int(0)
    th = int(threads) if threads else int(L.omp_default_threads())
    st = L.omp_pipecg(A.n, _p(rp), _p(ci), _p(val), _p(b), _p(x), float(tol), int(maxit), int(fixed_iters),
                      int(stop), th, ctypes.byref(it))
    if st < 0:
        raise ValueError("bad input to PIPECG-OpenMP")
    return x, st, it.value
