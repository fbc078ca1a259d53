"""Write tests/golden/c2_poisson3d_128_pcg.txt from the FP64 oracle only.

Workload: 3-D 7-point Poisson on a 128^3 grid, x* uniform in [-1, 1]
(seed 1), b = A x*, x0 = 0, Jacobi preconditioner.  Records, from the
oracle's Algorithm 1 (classic PCG):
  * x after exactly 500 iterations: its 2-norm and 4096 entries at indices
    drawn with default_rng(12345) (sampled, since the vector has 2^21 entries);
  * the iteration count and true relative residual of a solve to relative
    residual 1e-10.
Run from the repository root:  python tests/golden/make_c2_pcg_reference.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import poisson3d, rhs_from_solution, xstar_uniform  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_poisson3d_128_pcg.txt")


def main():
    A = poisson3d(128)
    b = rhs_from_solution(A, xstar_uniform(A.n, seed=1))
    t = time.time()
    r500 = oracle.pcg(A, b, fixed_iters=500)
    t500 = time.time() - t
    t = time.time()
    rtol = oracle.pcg(A, b, tol=1e-10, maxit=10000)
    ttol = time.time() - t
    idx = np.sort(np.random.default_rng(12345).choice(A.n, size=4096, replace=False))
    with open(OUT, "w") as f:
        f.write("# FP64 oracle (Algorithm 1, PCG, Jacobi) on 3-D 7-point Poisson 128^3,\n")
        f.write("# x* = U[-1,1] (default_rng(1)), b = A x*, x0 = 0.  Written by make_c2_pcg_reference.py.\n")
        f.write(f"# oracle time: 500 iterations {t500:.1f} s, tolerance solve {ttol:.1f} s\n")
        f.write(f"norm_x500 {np.linalg.norm(r500.x):.17e}\n")
        f.write(f"tol1e-10_iters {rtol.iters}\n")
        f.write(f"tol1e-10_status {rtol.status}\n")
        f.write(f"tol1e-10_rel_true {rtol.rel_true:.17e}\n")
        for i in idx:
            f.write(f"x500 {i} {r500.x[i]:.17e}\n")
    print(f"wrote {OUT}: iters to 1e-10 = {rtol.iters}, t500 = {t500:.1f}s")


if __name__ == "__main__":
    main()
