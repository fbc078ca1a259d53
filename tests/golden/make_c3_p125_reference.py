"""Write the full-size reference values of the 27-point and 125-point
workloads from the FP64 oracle only.

* c3_stencil27_160.txt -- 3-D 27-point lognormal stencil, 160^3 (seed 0,
  shift 1e-3), x* = U[-1,1] (seed 1), b = A x*, x0 = 0: x after exactly 10
  iterations of the oracle's Algorithm 2 (2-norm and 4096 sampled entries).
* p125_side165.txt -- 125-point Poisson, side 165 (Table 2's first size), the
  paper's protocol: x* = 1/sqrt(N), b = A x*, x0 = 0: x after exactly 5
  iterations (2-norm and 4096 sampled entries), and the iteration count of
  the absolute preconditioned-residual solve to 1e-5.
* c3_stencil27_160_x200.txt -- the same C3 system: x after exactly 200
  iterations, once with the oracle's dot products summed left to right
  (x200) and once with Neumaier's compensated sums (x200c).  The two differ
  only in the rounding of the dot products, so their distance measures how
  far any reordering of those sums moves the 200th iterate.
* c3_stencil27_160_tol.txt -- the same C3 system solved by the oracle's
  Algorithm 2 to a relative residual of 1e-10 (x_tol), with its iteration
  count, restarts and true relative residual, and ||b||.
Sample indices are drawn with default_rng(12345).  Run from the repository
root:  python tests/golden/make_c3_p125_reference.py [c3 c3_x200 c3_tol p125]
(no argument: all of them)
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import poisson125, rhs_from_solution, stencil27_lognormal, xstar_paper, xstar_uniform  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def write(path, header, meta, x, k, extra=()):
    """extra: further (key, vector) pairs sampled at the same indices."""
    idx = np.sort(np.random.default_rng(12345).choice(x.size, size=4096, replace=False))
    with open(path, "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        for key, v in meta.items():
            f.write(f"{key} {v}\n")
        f.write(f"norm_x{k} {np.linalg.norm(x):.17e}\n")
        for key, y in extra:
            f.write(f"norm_{key} {np.linalg.norm(y):.17e}\n")
        for i in idx:
            f.write(f"x{k} {i} {x[i]:.17e}\n")
        for key, y in extra:
            for i in idx:
                f.write(f"{key} {i} {y[i]:.17e}\n")


C3_HEAD = ["FP64 oracle (Algorithm 2, PIPECG, Jacobi) on the 27-point lognormal stencil 160^3 (seed 0, shift 1e-3),",
           "x* = U[-1,1] (default_rng(1)), b = A x*, x0 = 0.  Written by make_c3_p125_reference.py."]


def c3_system():
    A = stencil27_lognormal(160, seed=0, shift=1e-3)
    return A, rhs_from_solution(A, xstar_uniform(A.n, seed=1))


def c3_x200():
    A, b = c3_system()
    t = time.time()
    ra = oracle.pipecg(A, b, fixed_iters=200)
    ta = time.time() - t
    rc = oracle.pipecg(A, b, fixed_iters=200, dots="comp")
    sens = np.linalg.norm(rc.x - ra.x) / np.linalg.norm(ra.x)
    write(os.path.join(HERE, "c3_stencil27_160_x200.txt"),
          C3_HEAD + ["x200: dot products summed left to right; x200c: Neumaier-compensated dot products.",
                     f"oracle time for 200 iterations: {ta:.1f} s"],
          {"n": A.n, "nnz": A.nnz, "rel_diff_x200c_x200": f"{sens:.6e}"}, ra.x, 200, extra=[("x200c", rc.x)])


def c3_tol():
    A, b = c3_system()
    t = time.time()
    r = oracle.pipecg(A, b, tol=1e-10, maxit=20000)
    write(os.path.join(HERE, "c3_stencil27_160_tol.txt"),
          C3_HEAD + ["x_tol: the solve to relative residual 1e-10 (restarts from x when the true residual",
                     f"is above it).  Oracle time: {time.time() - t:.1f} s"],
          {"n": A.n, "nnz": A.nnz, "tol": 1e-10, "iters": r.iters, "restarts": r.restarts, "status": r.status,
           "rel_true": f"{r.rel_true:.17e}", "bnorm": f"{r.bnorm:.17e}"}, r.x, "_tol")


def c3_x10():
    A, b = c3_system()
    t = time.time()
    r = oracle.pipecg(A, b, fixed_iters=10)
    write(os.path.join(HERE, "c3_stencil27_160.txt"),
          C3_HEAD + [f"oracle time for 10 iterations: {time.time() - t:.1f} s"], {"n": A.n, "nnz": A.nnz}, r.x, 10)


def p125():
    A = poisson125(165)
    b = rhs_from_solution(A, xstar_paper(A.n))
    t = time.time()
    r5 = oracle.pipecg(A, b, fixed_iters=5)
    t5 = time.time() - t
    t = time.time()
    rp = oracle.pipecg(A, b, tol=1e-5, stop=oracle.STOP_ABS, maxit=10000)
    write(os.path.join(HERE, "p125_side165.txt"),
          ["FP64 oracle (Algorithm 2, PIPECG, Jacobi) on the 125-point Poisson matrix, side 165 (Table 2),",
           "x* = 1/sqrt(N), b = A x*, x0 = 0.  Written by make_c3_p125_reference.py.",
           f"oracle time: 5 iterations {t5:.1f} s, protocol solve {time.time() - t:.1f} s"],
          {"n": A.n, "nnz": A.nnz, "abs1e-5_iters": rp.iters, "abs1e-5_status": rp.status,
           "abs1e-5_precond_norm": f"{rp.precond_norm:.17e}"}, r5.x, 5)


def main(which):
    parts = {"c3": c3_x10, "c3_x200": c3_x200, "c3_tol": c3_tol, "p125": p125}
    for w in which or list(parts):
        parts[w]()
        print(f"{w} done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
