"""Thin ctypes binding of libppcg.so (include/ppcg.h).

Argument marshalling only: every step of a solve runs in the HIP library.
torch provides device memory and the stream; vectors are float64 CUDA
tensors.  If the library is not built this module raises at first use -- there
is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
# PPCG_LIB selects another build of the library (the tests' sanitized side build)
LIB_PATH = os.environ.get("PPCG_LIB") or os.path.join(HERE, "libppcg.so")

# ppcg_status
OK, NOT_CONVERGED, BREAKDOWN, STAGNATED = 0, 1, 2, 3
ERR_INVALID_ARG, ERR_BAD_CSR, ERR_NOMEM, ERR_DEVICE, ERR_BUDGET = -1, -2, -3, -4, -5
STOP_REL_RESID, STOP_PRECOND_ABS = 0, 1
FP64, MIXED_FP32, MIXED_FP32_VALUES, PRECISION_AUTO = 0, 1, 2, 3
MEM_DEVICE, MEM_HOST = 0, 1
METHOD_PIPECG, METHOD_PCG = 0, 1
FLAG_BORROW_INPUTS, FLAG_SELL_COL16, FLAG_SELL_COL32 = 1, 2, 4
FLAG_SELL_VALUE_TABLE, FLAG_SELL_FULL_VALUES = 8, 16
FLAG_ITER_FUSED, FLAG_ITER_TWO_LAUNCH = 32, 64
FLAG_SELL_SHARED_OFFSETS, FLAG_SELL_NO_SHARED_OFFSETS = 128, 256
SPMV_AUTO, SPMV_SELL, SPMV_CSR_VECTOR = 0, 1, 2

_STOP = {"rel": STOP_REL_RESID, "abs": STOP_PRECOND_ABS}
_PREC = {"fp64": FP64, "mixed": MIXED_FP32, "mixed_values": MIXED_FP32_VALUES, "auto": PRECISION_AUTO}
_FMT = {"auto": SPMV_AUTO, "sell": SPMV_SELL, "csr_vector": SPMV_CSR_VECTOR}
_METHOD = {"pipecg": METHOD_PIPECG, "pcg": METHOD_PCG}


class Csr(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("mem", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("max_restarts", ctypes.c_int32), ("stop", ctypes.c_int),
                ("precision", ctypes.c_int), ("vec_mem", ctypes.c_int), ("spmv_format", ctypes.c_int),
                ("graph_iters", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("method", ctypes.c_int), ("flags", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("status", ctypes.c_int), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_resid_true", ctypes.c_double), ("rel_resid_recur", ctypes.c_double),
                ("precond_norm", ctypes.c_double), ("time_ms", ctypes.c_double), ("model_bytes", ctypes.c_double),
                ("precision", ctypes.c_int), ("method", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class MatrixInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("nnz_stored", ctypes.c_int64), ("format", ctypes.c_int), ("sell_c", ctypes.c_int32),
                ("sell_sigma", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("bytes_per_iter", ctypes.c_double), ("bytes_vma", ctypes.c_double),
                ("bytes_spmv", ctypes.c_double), ("device_bytes", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("col_index_bytes", ctypes.c_int32), ("diag_const", ctypes.c_int32),
                ("value_bytes", ctypes.c_int32), ("distinct_values", ctypes.c_int32),
                ("iter_launches", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class ShardInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("row_begin", ctypes.c_int32), ("row_end", ctypes.c_int32),
                ("nnz_local", ctypes.c_int64), ("nnz_remote", ctypes.c_int64), ("halo", ctypes.c_int32),
                ("boundary_rows", ctypes.c_int32), ("bytes_part1", ctypes.c_double),
                ("bytes_part2", ctypes.c_double), ("halo_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class HybridInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("n_cpu", ctypes.c_int32), ("n_gpu", ctypes.c_int32),
                ("host_threads", ctypes.c_int32), ("t_cpu_spmv_ms", ctypes.c_double),
                ("t_gpu_spmv_ms", ctypes.c_double), ("nnz_cpu_local", ctypes.c_int64),
                ("nnz_cpu_remote", ctypes.c_int64), ("nnz_gpu_local", ctypes.c_int64),
                ("nnz_gpu_remote", ctypes.c_int64), ("halo_to_cpu", ctypes.c_int32), ("halo_to_gpu", ctypes.c_int32),
                ("scheme", ctypes.c_int), ("copy_bytes_per_iter", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


EXPORTS = ["ppcg_default_options", "ppcg_create", "ppcg_set_options", "ppcg_solve", "ppcg_solve_batch",
           "ppcg_spmv",
           "ppcg_get_matrix_info", "ppcg_footprint_bytes", "ppcg_time_kernels", "ppcg_destroy",
           "ppcg_status_str", "ppcg_last_error", "ppcg_split_rows", "ppcg_shard_create", "ppcg_shard_get_info",
           "ppcg_shard_halo_columns", "ppcg_shard_gather", "ppcg_shard_spmv", "ppcg_shard_time",
           "ppcg_shard_destroy", "ppcg_hybrid_create", "ppcg_hybrid_get_info", "ppcg_hybrid_solve",
           "ppcg_hybrid_destroy", "ppcg_srv_create", "ppcg_srv_submit", "ppcg_srv_step",
           "ppcg_srv_poll", "ppcg_srv_destroy", "ppcg_solve_noalloc"]

_lib = None


def lib():
    """Load libppcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2105_06176_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ppcg_default_options": ([ctypes.POINTER(Options)], ctypes.c_int),
        "ppcg_create": ([ctypes.POINTER(Csr), ctypes.POINTER(Options), P, ctypes.POINTER(P)], ctypes.c_int),
        "ppcg_set_options": ([P, ctypes.POINTER(Options)], ctypes.c_int),
        "ppcg_solve": ([P, P, P, P, ctypes.POINTER(Info)], ctypes.c_int),
        "ppcg_solve_batch": ([I32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                              ctypes.POINTER(Info)], ctypes.c_int),
        "ppcg_spmv": ([P, P, P], ctypes.c_int),
        "ppcg_get_matrix_info": ([P, ctypes.POINTER(MatrixInfo)], ctypes.c_int),
        "ppcg_footprint_bytes": ([I32, I64, ctypes.c_int], D),
        "ppcg_time_kernels": ([P, P, I32, ctypes.POINTER(D), ctypes.POINTER(D)], ctypes.c_int),
        "ppcg_destroy": ([P], ctypes.c_int),
        "ppcg_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "ppcg_last_error": ([], ctypes.c_char_p),
        "ppcg_split_rows": ([I32, P, I32, P, P], ctypes.c_int),
        "ppcg_shard_create": ([ctypes.POINTER(Csr), I32, I32, P, ctypes.POINTER(P)], ctypes.c_int),
        "ppcg_shard_get_info": ([P, ctypes.POINTER(ShardInfo)], ctypes.c_int),
        "ppcg_shard_halo_columns": ([P, P], ctypes.c_int),
        "ppcg_shard_gather": ([P, P, P], ctypes.c_int),
        "ppcg_shard_spmv": ([P, P, P, P, I32], ctypes.c_int),
        "ppcg_shard_time": ([P, P, P, P, P, I32, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)],
                            ctypes.c_int),
        "ppcg_shard_destroy": ([P], ctypes.c_int),
        "ppcg_hybrid_create": ([ctypes.POINTER(Csr), ctypes.POINTER(Options), ctypes.c_int, I32, D, P,
                                ctypes.POINTER(P)], ctypes.c_int),
        "ppcg_hybrid_get_info": ([P, ctypes.POINTER(HybridInfo)], ctypes.c_int),
        "ppcg_hybrid_solve": ([P, P, P, P, ctypes.POINTER(Info)], ctypes.c_int),
        "ppcg_hybrid_destroy": ([P], ctypes.c_int),
        "ppcg_srv_create": ([ctypes.POINTER(Options), D, ctypes.POINTER(P)], ctypes.c_int),
        "ppcg_srv_submit": ([P, ctypes.POINTER(Csr), P, D, ctypes.c_int, ctypes.POINTER(I64)], ctypes.c_int),
        "ppcg_srv_step": ([P, ctypes.POINTER(I32), ctypes.POINTER(I32)], ctypes.c_int),
        "ppcg_srv_poll": ([P, I64, ctypes.POINTER(I32), P, ctypes.POINTER(Info)], ctypes.c_int),
        "ppcg_srv_destroy": ([P], ctypes.c_int),
        "ppcg_solve_noalloc": ([ctypes.POINTER(Csr), ctypes.POINTER(Options), P, P, P, ctypes.POINTER(Info), P],
                               ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class PPCGError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        self.status = status
        msg = L.ppcg_last_error().decode()
        super().__init__(f"{where}: {L.ppcg_status_str(status).decode()} {msg}")


def _check(status: int, where: str) -> int:
    if status < 0:
        raise PPCGError(status, where)
    return status


def _stream_ptr(stream) -> Optional[int]:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def make_options(**kw) -> Options:
    o = Options()
    _check(lib().ppcg_default_options(ctypes.byref(o)), "ppcg_default_options")
    for k, v in kw.items():
        if k == "stop":
            v = _STOP.get(v, v)
        elif k == "precision":
            v = _PREC.get(v, v)
        elif k == "spmv_format":
            v = _FMT.get(v, v)
        elif k == "method":
            v = _METHOD.get(v, v)
        elif k == "vec_mem":
            v = {"device": MEM_DEVICE, "host": MEM_HOST}.get(v, v)
        setattr(o, k, v)
    return o


def _csr_struct(A, keep: list) -> Csr:
    """Describe A for the ABI: a workloads.CSR (host numpy) or a tuple of CUDA
    tensors (row_ptr int32, col_idx int32, values float64)."""
    import numpy as np

    c = Csr()
    c.struct_size = ctypes.sizeof(Csr)
    if isinstance(A, tuple):
        rp, ci, val = A
        c.n = int(rp.numel() - 1)
        c.nnz = int(ci.numel())
        c.row_ptr, c.col_idx, c.values = rp.data_ptr(), ci.data_ptr(), val.data_ptr()
        c.mem = MEM_HOST if rp.device.type == "cpu" else MEM_DEVICE
        keep.extend([rp, ci, val])
    else:
        rp = np.ascontiguousarray(A.rp, dtype=np.int32)
        ci = np.ascontiguousarray(A.ci, dtype=np.int32)
        val = np.ascontiguousarray(A.val, dtype=np.float64)
        keep.extend([rp, ci, val])
        c.n = int(A.n)
        c.nnz = int(ci.size)
        c.row_ptr, c.col_idx, c.values = rp.ctypes.data, ci.ctypes.data, val.ctypes.data
        c.mem = MEM_HOST
    return c


def _vec_ptr(t, n: int, name: str):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 tensor of {n} elements")
    return t.data_ptr()


class Solver:
    """One sparse SPD matrix prepared for PIPECG solves (ppcg_create)."""

    def __init__(self, A, stream=None, **options):
        self._keep: list = []
        self.opt = make_options(**options)
        c = _csr_struct(A, self._keep)
        self.n = int(c.n)
        h = ctypes.c_void_p()
        _check(lib().ppcg_create(ctypes.byref(c), ctypes.byref(self.opt), _stream_ptr(stream), ctypes.byref(h)),
               "ppcg_create")
        self._keep = []
        self.h = h
        self.stream = stream

    def set_options(self, **options):
        self.opt = make_options(**options)
        _check(lib().ppcg_set_options(self.h, ctypes.byref(self.opt)), "ppcg_set_options")

    def _alloc(self):
        import torch

        return torch.empty(self.n, dtype=torch.float64, device="cuda")

    def solve(self, b, x0=None, out=None) -> Tuple[object, dict]:
        x = out if out is not None else self._alloc()
        info = Info()
        info.struct_size = ctypes.sizeof(Info)
        st = lib().ppcg_solve(self.h, _vec_ptr(b, self.n, "b"), _vec_ptr(x0, self.n, "x0"),
                              _vec_ptr(x, self.n, "x"), ctypes.byref(info))
        _check(st, "ppcg_solve")
        return x, info.as_dict()

    def spmv(self, x, out=None):
        y = out if out is not None else self._alloc()
        _check(lib().ppcg_spmv(self.h, _vec_ptr(x, self.n, "x"), _vec_ptr(y, self.n, "y")), "ppcg_spmv")
        return y

    def matrix_info(self) -> dict:
        mi = MatrixInfo()
        mi.struct_size = ctypes.sizeof(MatrixInfo)
        _check(lib().ppcg_get_matrix_info(self.h, ctypes.byref(mi)), "ppcg_get_matrix_info")
        return mi.as_dict()

    def time_kernels(self, b, iters: int = 20) -> Tuple[float, float]:
        a, s = ctypes.c_double(), ctypes.c_double()
        _check(lib().ppcg_time_kernels(self.h, _vec_ptr(b, self.n, "b"), iters, ctypes.byref(a), ctypes.byref(s)),
               "ppcg_time_kernels")
        return a.value, s.value

    def close(self):
        if getattr(self, "h", None):
            lib().ppcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers: Sequence[Solver], bs: Sequence, x0s: Optional[Sequence] = None,
                outs: Optional[Sequence] = None) -> Tuple[List, List[dict]]:
    n = len(solvers)
    xs = list(outs) if outs is not None else [s._alloc() for s in solvers]
    arr = ctypes.c_void_p * n
    hs = arr(*[s.h.value for s in solvers])
    bp = arr(*[_vec_ptr(b, s.n, "b") for s, b in zip(solvers, bs)])
    xp = arr(*[_vec_ptr(x, s.n, "x") for s, x in zip(solvers, xs)])
    x0p = arr(*[_vec_ptr(x0, s.n, "x0") for s, x0 in zip(solvers, x0s)]) if x0s is not None else None
    infos = (Info * n)()
    for i in range(n):
        infos[i].struct_size = ctypes.sizeof(Info)
    _check(lib().ppcg_solve_batch(n, hs, bp, x0p, xp, infos), "ppcg_solve_batch")
    return xs, [infos[i].as_dict() for i in range(n)]


def solve_noalloc(A, b, x0=None, out=None, stream=None, **options) -> Tuple[object, dict]:
    """ppcg_solve_noalloc: A is a tuple of CUDA tensors (row_ptr int32,
    col_idx int32, values float64); b, x0, out float64 CUDA tensors.  The
    library allocates nothing; out (allocated here when not given) receives x."""
    import torch

    keep: list = []
    c = _csr_struct(A, keep)
    n = int(c.n)
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device="cuda")
    opt = make_options(**options)
    info = Info()
    info.struct_size = ctypes.sizeof(Info)
    st = lib().ppcg_solve_noalloc(ctypes.byref(c), ctypes.byref(opt), _vec_ptr(b, n, "b"), _vec_ptr(x0, n, "x0"),
                                  _vec_ptr(x, n, "x"), ctypes.byref(info), _stream_ptr(stream))
    _check(st, "ppcg_solve_noalloc")
    return x, info.as_dict()


def footprint_bytes(n: int, nnz: int, precision: str = "fp64") -> float:
    return lib().ppcg_footprint_bytes(n, nnz, _PREC[precision])


class Server:
    """Continuous-batching solve server (ppcg_srv_*)."""

    def __init__(self, budget_bytes: float = 0.0, borrow: bool = False, **options):
        """borrow: requests reference the submitted arrays (kept alive here
        until polled ready) instead of the server copying them."""
        if borrow:
            options["flags"] = options.get("flags", 0) | FLAG_BORROW_INPUTS
        self.opt = make_options(**options)
        s = ctypes.c_void_p()
        _check(lib().ppcg_srv_create(ctypes.byref(self.opt), float(budget_bytes), ctypes.byref(s)),
               "ppcg_srv_create")
        self.s = s
        self._n = {}
        self._borrowed = {}

    def submit(self, A, b, tol: float, precision: str = "fp64") -> int:
        import numpy as np

        keep: list = []
        c = _csr_struct(A, keep)
        if c.mem != MEM_HOST:
            raise ValueError("server requests take host CSR arrays")
        bb = np.ascontiguousarray(b, dtype=np.float64)
        rid = ctypes.c_int64()
        _check(lib().ppcg_srv_submit(self.s, ctypes.byref(c), bb.ctypes.data, float(tol), _PREC[precision],
                                     ctypes.byref(rid)), "ppcg_srv_submit")
        self._n[rid.value] = int(c.n)
        if self.opt.flags & FLAG_BORROW_INPUTS:
            self._borrowed[rid.value] = (keep, bb)
        return rid.value

    def step(self) -> Tuple[int, int]:
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ppcg_srv_step(self.s, ctypes.byref(a), ctypes.byref(q)), "ppcg_srv_step")
        return a.value, q.value

    def poll(self, rid: int):
        import numpy as np

        ready = ctypes.c_int32()
        x = np.empty(self._n[rid], dtype=np.float64)
        info = Info()
        info.struct_size = ctypes.sizeof(Info)
        st = lib().ppcg_srv_poll(self.s, rid, ctypes.byref(ready), x.ctypes.data, ctypes.byref(info))
        _check(st, "ppcg_srv_poll")
        if not ready.value:
            return None
        del self._n[rid]
        self._borrowed.pop(rid, None)
        return x, info.as_dict()

    def close(self):
        if getattr(self, "s", None):
            lib().ppcg_srv_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_rows(row_ptr, times) -> List[int]:
    """Row boundaries of the performance-model split (host only, no GPU)."""
    import numpy as np

    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    t = np.ascontiguousarray(times, dtype=np.float64)
    out = np.zeros(len(t) + 1, dtype=np.int32)
    _check(lib().ppcg_split_rows(int(rp.size - 1), rp.ctypes.data, int(t.size), t.ctypes.data, out.ctypes.data),
           "ppcg_split_rows")
    return [int(v) for v in out]


class Shard:
    """One unit's rows of A under the 2-D decomposition (part 1 local columns,
    part 2 halo columns)."""

    def __init__(self, A, row_begin: int, row_end: int, stream=None):
        keep: list = []
        c = _csr_struct(A, keep)
        s = ctypes.c_void_p()
        _check(lib().ppcg_shard_create(ctypes.byref(c), int(row_begin), int(row_end), _stream_ptr(stream),
                                       ctypes.byref(s)), "ppcg_shard_create")
        self.s = s
        self.rows = int(row_end - row_begin)

    def info(self) -> dict:
        i = ShardInfo()
        i.struct_size = ctypes.sizeof(ShardInfo)
        _check(lib().ppcg_shard_get_info(self.s, ctypes.byref(i)), "ppcg_shard_get_info")
        return i.as_dict()

    def halo_columns(self):
        import numpy as np

        h = self.info()["halo"]
        cols = np.zeros(max(h, 1), dtype=np.int32)
        _check(lib().ppcg_shard_halo_columns(self.s, cols.ctypes.data), "ppcg_shard_halo_columns")
        return cols[:h]

    def gather(self, x_global, x_halo):
        _check(lib().ppcg_shard_gather(self.s, x_global.data_ptr(), x_halo.data_ptr()), "ppcg_shard_gather")

    def spmv(self, x_local, x_halo, y, parts: int = 3):
        xh = x_halo.data_ptr() if x_halo is not None else None
        _check(lib().ppcg_shard_spmv(self.s, x_local.data_ptr(), xh, y.data_ptr(), int(parts)), "ppcg_shard_spmv")
        return y

    def time(self, x_global, x_local, x_halo, y, iters: int = 50) -> Tuple[float, float, float]:
        a, g, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().ppcg_shard_time(self.s, x_global.data_ptr(), x_local.data_ptr(), x_halo.data_ptr(),
                                     y.data_ptr(), int(iters), ctypes.byref(a), ctypes.byref(g), ctypes.byref(c)),
               "ppcg_shard_time")
        return a.value, g.value, c.value

    def close(self):
        if getattr(self, "s", None):
            lib().ppcg_shard_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hybrid:
    """Algorithm 2 on host threads and the GPU together.  scheme 3 (default):
    rows split by the performance model, or by a forced share of the
    non-zeros; schemes 1 and 2: every row on the GPU, dot products (and for 2
    the vector updates) repeated on the host."""

    def __init__(self, A, host_threads: int = 4, cpu_share: float = -1.0, stream=None, scheme: int = 3,
                 **options):
        options.setdefault("vec_mem", "host")
        self.opt = make_options(**options)
        keep: list = []
        c = _csr_struct(A, keep)
        if c.mem != MEM_HOST:
            raise ValueError("the host + GPU solver takes host CSR arrays")
        h = ctypes.c_void_p()
        _check(lib().ppcg_hybrid_create(ctypes.byref(c), ctypes.byref(self.opt), int(scheme), int(host_threads),
                                        float(cpu_share), _stream_ptr(stream), ctypes.byref(h)),
               "ppcg_hybrid_create")
        self.h = h
        self.n = int(c.n)

    def info(self) -> dict:
        i = HybridInfo()
        i.struct_size = ctypes.sizeof(HybridInfo)
        _check(lib().ppcg_hybrid_get_info(self.h, ctypes.byref(i)), "ppcg_hybrid_get_info")
        return i.as_dict()

    def solve(self, b, x0=None):
        import numpy as np

        bb = np.ascontiguousarray(b, dtype=np.float64)
        xx = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        x = np.empty(self.n, dtype=np.float64)
        info = Info()
        info.struct_size = ctypes.sizeof(Info)
        _check(lib().ppcg_hybrid_solve(self.h, bb.ctypes.data, None if xx is None else xx.ctypes.data,
                                       x.ctypes.data, ctypes.byref(info)), "ppcg_hybrid_solve")
        return x, info.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().ppcg_hybrid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
