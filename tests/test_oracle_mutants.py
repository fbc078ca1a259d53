"""Strength of the oracle's pins.

Each mutant is one plausible mistake planted in a copy of the oracle's C
source -- a dropped term, a flipped sign, a wrong index or a swapped operand
in Algorithm 1, Algorithm 2, the SpMV, the Jacobi preconditioner, a dot
product or the stopping test.  The copy is compiled on the CPU and loaded in
place of the oracle (ORACLE_LIB); the pin suite must then fail.  The mistake
is planted in the copy only: the oracle itself is never modified.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ppcg_oracle.c")

# (name, original text, mutated text, which occurrence of the original: 0-based)
MUTANTS = [
    ("spmv reads x at the row index", "double prod = v[k] * x[ci[k]];", "double prod = v[k] * x[i];", 0),
    ("compensated dot squares its first operand", "double prod = a[i] * b[i];", "double prod = a[i] * a[i];", 0),
    ("dot product squares its first operand", "double prod = a[i] * b[i];", "double prod = a[i] * a[i];", 1),
    ("compensated dot drops its correction", "return acc + comp;", "return acc;", 0),
    ("compensated dot takes the wrong branch's error", "comp = comp + ((acc - t) + prod);",
     "comp = comp + ((prod - t) + acc);", 0),
    ("Jacobi applies a_ii instead of its inverse", "dinv[i] = 1.0 / d;", "dinv[i] = d;", 0),
    ("stopping test uses the preconditioned residual", "return sqrt(rr) <= tol * bnorm;",
     "return sqrt(uu) <= tol * bnorm;", 0),
    ("PCG beta inverted", "double beta = i > 0 ? gamma / gamma_prev : 0.0;",
     "double beta = i > 0 ? gamma_prev / gamma : 0.0;", 0),
    # (s, u) would be an equivalent mutant: (A p, u) = (A p, p) by A-conjugacy of the directions
    ("PCG delta = (p, p)", "double delta = ora_dot(n, s, p);", "double delta = ora_dot(n, p, p);", 0),
    ("PCG preconditioner dropped in the loop", "u[k] = dinv[k] * r[k];", "u[k] = r[k];", 0),
    ("PCG x updated along s", "x[k] = x[k] + alpha * p[k];", "x[k] = x[k] + alpha * s[k];", 0),
    ("PIPECG z drops beta z", "z[k] = nv[k] + beta * z[k];", "z[k] = nv[k];", 0),
    ("PIPECG q with a minus sign", "q[k] = m[k] + beta * q[k];", "q[k] = m[k] - beta * q[k];", 0),
    ("PIPECG s recurs on p", "s[k] = w[k] + beta * s[k];", "s[k] = w[k] + beta * p[k];", 0),
    ("PIPECG p drops beta p", "p[k] = u[k] + beta * p[k];", "p[k] = u[k];", 1),
    ("PIPECG x updated along s", "x[k] = x[k] + alpha * p[k];", "x[k] = x[k] + alpha * s[k];", 1),
    ("PIPECG r with a plus sign", "r[k] = r[k] - alpha * s[k];", "r[k] = r[k] + alpha * s[k];", 1),
    ("PIPECG u updated along z", "u[k] = u[k] - alpha * q[k];", "u[k] = u[k] - alpha * z[k];", 0),
    ("PIPECG w updated along q", "w[k] = w[k] - alpha * z[k];", "w[k] = w[k] - alpha * q[k];", 0),
    ("PIPECG alpha denominator sign", "denom = delta - beta * gamma / alpha_prev;",
     "denom = delta + beta * gamma / alpha_prev;", 0),
    ("PIPECG delta from (w, r)", "delta = ora_dot(n, w, u);", "delta = ora_dot(n, w, r);", 1),
    ("PIPECG m without the preconditioner", "m[k] = dinv[k] * w[k];", "m[k] = w[k];", 0),
    ("PIPECG w0 = A r0 instead of A u0", "ora_spmv(n, rp, ci, v, u, w);", "ora_spmv(n, rp, ci, v, r, w);", 0),
]


def _replace_nth(text, old, new, k):
    start = -1
    for _ in range(k + 1):
        start = text.find(old, start + 1)
        assert start >= 0, f"mutation site not found: {old!r} (occurrence {k})"
    return text[:start] + new + text[start + len(old):]


@pytest.mark.parametrize("name,old,new,k", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, k):
    src = open(SRC).read()
    mutant = _replace_nth(src, old, new, k)
    assert mutant != src
    c = tmp_path / "mutant.c"
    c.write_text(mutant)
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o",
                    str(so), str(c), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"no pin fails for the mutant '{name}':\n{r.stdout[-2000:]}"


PART = os.path.join(ROOT, "oracle", "partition.py")

PARTITION_MUTANTS = [
    ("unit may exceed its share", "while k < len(rp) - 1 and rp[k + 1] <= nnz_target:",
     "while k < len(rp) - 1 and rp[k] <= nnz_target:", 0),
    ("shares not cumulative", "        cum += r[k]\n", "        cum = r[k]\n", 0),
    ("speed taken as time", "s = [nnz / float(t) for t in times]", "s = [float(t) for t in times]", 0),
    ("last local column counted remote", "if lo <= c < hi:\n                nnz1 += 1",
     "if lo <= c < hi - 1:\n                nnz1 += 1", 0),
    ("part 2 dropped from the split product", "y[i - lo] = p1 + p2", "y[i - lo] = p1", 0),
]


@pytest.mark.parametrize("name,old,new,k", PARTITION_MUTANTS, ids=[m[0] for m in PARTITION_MUTANTS])
def test_partition_pins_catch_planted_mistake(tmp_path, name, old, new, k):
    src = open(PART).read()
    mutant = _replace_nth(src, old, new, k)
    assert mutant != src
    f = tmp_path / "partition_mutant.py"
    f.write_text(mutant)
    env = dict(os.environ, ORACLE_PARTITION=str(f))
    # the pins alone: the comparisons with the library are left out
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-k", "not library",
                        os.path.join(ROOT, "tests", "test_partition_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"no pin fails for the mutant '{name}':\n{r.stdout[-2000:]}"
