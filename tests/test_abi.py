"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ppcg.h declares, and the ctypes mirrors of the ABI
structs have the C layout."""

import ctypes
import os
import re
import subprocess

import pytest

from paper_2105_06176_amd import ppcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppcg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ppcg_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(ppcg.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    L = ppcg.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_header_flag_values_match_the_binding():
    src = open(HEADER).read()
    flags = dict(re.findall(r"#define PPCG_FLAG_([A-Z0-9_]+) (\d+)u", src))
    assert flags and set(flags) == {k[5:] for k in dir(ppcg) if k.startswith("FLAG_")}
    for name, v in flags.items():
        assert getattr(ppcg, "FLAG_" + name) == int(v), name
    bits = [int(v) for v in flags.values()]
    assert len(set(bits)) == len(bits) and all(b & (b - 1) == 0 for b in bits)


def test_default_options_and_status_strings():
    o = ppcg.make_options()
    assert o.struct_size == ctypes.sizeof(ppcg.Options)
    assert o.tol == 1e-8 and o.max_iter == 10000 and o.max_restarts == 3
    L = ppcg.lib()
    assert L.ppcg_status_str(ppcg.OK) == b"PPCG_OK"
    assert L.ppcg_status_str(ppcg.ERR_BAD_CSR) == b"PPCG_ERR_BAD_CSR"


def test_host_side_argument_errors():
    L = ppcg.lib()
    assert L.ppcg_default_options(None) == ppcg.ERR_INVALID_ARG
    assert b"NULL" in L.ppcg_last_error()
    h = ctypes.c_void_p()
    o = ppcg.make_options()
    assert L.ppcg_create(None, ctypes.byref(o), None, ctypes.byref(h)) == ppcg.ERR_INVALID_ARG
    assert h.value is None
    bad = ppcg.make_options(tol=-1.0)
    c = ppcg.Csr()
    c.struct_size = ctypes.sizeof(ppcg.Csr)
    assert L.ppcg_create(ctypes.byref(c), ctypes.byref(bad), None, ctypes.byref(h)) == ppcg.ERR_INVALID_ARG
    assert L.ppcg_solve(None, None, None, None, None) == ppcg.ERR_INVALID_ARG
    assert L.ppcg_destroy(None) == ppcg.OK
    assert L.ppcg_srv_destroy(None) == ppcg.OK
    assert L.ppcg_shard_destroy(None) == ppcg.OK
    assert L.ppcg_hybrid_destroy(None) == ppcg.OK
    assert L.ppcg_hybrid_create(None, None, 3, 1, -1.0, None, None) == ppcg.ERR_INVALID_ARG
    assert L.ppcg_shard_create(None, 0, 1, None, None) == ppcg.ERR_INVALID_ARG
    assert L.ppcg_footprint_bytes(0, 0, 0) == 0.0
    assert L.ppcg_footprint_bytes(1000, 5000, 1) > L.ppcg_footprint_bytes(1000, 5000, 0) > 0


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "ppcg.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("ppcg_csr %zu\nppcg_options %zu\nppcg_info %zu\nppcg_matrix_info %zu\n",
         sizeof(ppcg_csr), sizeof(ppcg_options), sizeof(ppcg_info), sizeof(ppcg_matrix_info));
  printf("ppcg_shard_info %zu\nppcg_hybrid_info %zu\n", sizeof(ppcg_shard_info), sizeof(ppcg_hybrid_info));
  F(ppcg_csr, nnz) F(ppcg_csr, values) F(ppcg_csr, mem)
  F(ppcg_options, tol) F(ppcg_options, stop) F(ppcg_options, inner_tol) F(ppcg_options, method)
  F(ppcg_options, flags)
  F(ppcg_shard_info, nnz_local) F(ppcg_shard_info, boundary_rows) F(ppcg_shard_info, halo_bytes)
  F(ppcg_hybrid_info, t_cpu_spmv_ms) F(ppcg_hybrid_info, nnz_gpu_remote) F(ppcg_hybrid_info, halo_to_gpu)
  F(ppcg_hybrid_info, scheme) F(ppcg_hybrid_info, copy_bytes_per_iter)
  F(ppcg_info, status) F(ppcg_info, rel_resid_true) F(ppcg_info, model_bytes)
  F(ppcg_info, precision) F(ppcg_info, method)
  F(ppcg_matrix_info, nnz_stored) F(ppcg_matrix_info, tile_rows) F(ppcg_matrix_info, setup_ms)
  F(ppcg_matrix_info, col_index_bytes) F(ppcg_matrix_info, diag_const)
  F(ppcg_matrix_info, value_bytes) F(ppcg_matrix_info, distinct_values)
  return 0;
}
"""


def test_ctypes_structs_match_c_layout(tmp_path):
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text(LAYOUT_C)
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split() for line in out if line.strip())
    py = {"ppcg_csr": ppcg.Csr, "ppcg_options": ppcg.Options, "ppcg_info": ppcg.Info,
          "ppcg_matrix_info": ppcg.MatrixInfo, "ppcg_shard_info": ppcg.ShardInfo,
          "ppcg_hybrid_info": ppcg.HybridInfo}
    for k, v in got.items():
        if "." in k:
            t, m = k.split(".")
            assert getattr(py[t], m).offset == int(v), k
        else:
            assert ctypes.sizeof(py[k]) == int(v), k
