"""CPU-only sanitizer runs.  The oracle is rebuilt with AddressSanitizer and
UndefinedBehaviorSanitizer and its pin suite is run against that build; the
library's host code (argument checks, the row-split planner, the ABI
surface, everything that runs before a device is touched) is rebuilt with
both sanitizers on the host pass and the CPU ABI and split tests are run
against it.  Each run is a subprocess with the sanitizer runtime preloaded;
any finding aborts it, so the test fails."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Host-side AddressSanitizer + UndefinedBehaviorSanitizer for the HIP
# sources: each flag applies to the host pass alone (-Xarch_host).
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(env_extra, args):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip(f"{name} not available")
    return p


def test_oracle_pins_under_asan_ubsan(tmp_path):
    from oracle import build as ob

    lib = ob.build_sanitized(str(tmp_path / "liboracle_san.so"))
    pre = " ".join(_gcc_runtime(n) for n in ("libasan.so", "libubsan.so"))
    _run({"PPCG_ORACLE_LIB": lib, "LD_PRELOAD": pre}, ["tests/test_oracle_pins.py"])


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2105_06176_amd import build as lb

    rt = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang ASan runtime not available")
    lib = lb.build(extra_flags=["-O1", "-g", *HOST_SANITIZE], link_flags=HOST_SANITIZE,
                   out=str(tmp_path / "libppcg_san.so"))
    _run({"PPCG_LIB": lib, "LD_PRELOAD": rt[0]},
         ["tests/test_abi.py", "tests/test_partition_pins.py", "tests/test_contract.py"])
