"""Host-side checks of the product's contract (no GPU needed): the product
path has no CPU fallback and never touches the oracle, and bench.py runs on
one GPU only."""

import os
import subprocess
import sys

import pytest

from paper_2105_06176_amd import ppcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(ppcg, "_lib", None)
    monkeypatch.setattr(ppcg, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libppcg.so"))
    with pytest.raises(RuntimeError, match="missing"):
        ppcg.lib()
    with pytest.raises(RuntimeError, match="missing"):
        ppcg.make_options()


def test_product_package_does_not_load_the_oracle():
    code = ("import sys; import paper_2105_06176_amd, paper_2105_06176_amd.ppcg as p; p.lib(); "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "False"
    pkg = os.path.join(ROOT, "paper_2105_06176_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert "import oracle" not in src and "from oracle" not in src and "liboracle" not in src, f


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
