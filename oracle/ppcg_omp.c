/*
 * ppcg_omp.c -- the paper's CPU baseline, "PIPECG-OpenMP": Algorithm 2
 * (PIPECG, Section III-B) with the Jacobi preconditioner on host threads.
 *
 * TEST INFRASTRUCTURE ONLY (timing).  Like ppcg_oracle.c it is used by the
 * tests and by the benchmark's CPU baseline leg, never by the product path,
 * and shares no code with the HIP library.  It is not the checker: its dot
 * products are summed per thread and then across threads (OpenMP reduction
 * order), so its iterates differ from the sequential oracle by rounding; the
 * CPU tests hold it to the oracle within the 1e-10 bar.
 *
 * What the paper describes for its CPU implementation (Section V-A: every
 * PIPECG kernel with OpenMP; Section V-B "CPU related optimization": the
 * loops of the vector updates merged, so that each vector is brought into
 * the cache once per iteration):
 *   - one parallel loop per iteration for the eight vector updates of
 *     Algorithm 2, the Jacobi preconditioner m = M^-1 w (elementwise, so it
 *     joins the same loop) and the dot products gamma = (r,u), delta = (w,u)
 *     and (u,u), (r,r) as reductions;
 *   - one parallel loop for the SpMV n = A m (CSR, each row in stored order);
 *   - alpha and beta on one thread between them.
 * Stopping test at the top of the loop as in the oracle: sqrt((u,u)) < tol
 * (stop = 1) or sqrt((r,r)) <= tol ||b|| (stop = 0); fixed_iters > 0 runs
 * exactly that many iterations.  No restarts (the paper's method has none).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>

enum { OMP_OK = 0, OMP_NOT_CONVERGED = 1, OMP_BREAKDOWN = 2, OMP_BAD = -1 };

static void spmv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            acc = acc + v[k] * x[ci[k]];
        y[i] = acc;
    }
}

/* Returns the status; *iters_out receives the x-updates performed. */
int omp_pipecg(int n, const int *rp, const int *ci, const double *val, const double *b, double *x, double tol,
               int maxit, int fixed_iters, int stop, int threads, int *iters_out)
{
    if (n < 1 || !rp || !ci || !val || !b || !x || threads < 1)
        return OMP_BAD;
    omp_set_num_threads(threads);
    double *buf = malloc(sizeof(double) * (size_t)n * 11);
    if (!buf)
        return OMP_BAD;
    double *dinv = buf, *r = buf + (size_t)n, *u = buf + 2 * (size_t)n, *w = buf + 3 * (size_t)n;
    double *m = buf + 4 * (size_t)n, *nv = buf + 5 * (size_t)n, *z = buf + 6 * (size_t)n;
    double *q = buf + 7 * (size_t)n, *s = buf + 8 * (size_t)n, *p = buf + 9 * (size_t)n;
    double *t = buf + 10 * (size_t)n;
    int status = OMP_OK;
    /* Jacobi inverse diagonal, r = b - A x, u = M^-1 r */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i)
                d = val[k];
        dinv[i] = 1.0 / d;
    }
    spmv(n, rp, ci, val, x, t);
    double bb = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : bb)
    for (int i = 0; i < n; ++i) {
        r[i] = b[i] - t[i];
        u[i] = dinv[i] * r[i];
        z[i] = q[i] = s[i] = p[i] = 0.0;
        bb += b[i] * b[i];
    }
    spmv(n, rp, ci, val, u, w);
    double gamma = 0.0, delta = 0.0, uu = 0.0, rr = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : gamma, delta, uu, rr)
    for (int i = 0; i < n; ++i) {
        m[i] = dinv[i] * w[i];
        gamma += r[i] * u[i];
        delta += w[i] * u[i];
        uu += u[i] * u[i];
        rr += r[i] * r[i];
    }
    spmv(n, rp, ci, val, m, nv);
    const double bnorm = sqrt(bb);
    double gamma_old = 0.0, alpha_old = 0.0;
    int it = 0;
    for (;;) {
        if (fixed_iters > 0) {
            if (it >= fixed_iters || gamma == 0.0)
                break;
        } else {
            const int conv = stop == 1 ? sqrt(uu) < tol : sqrt(rr) <= tol * bnorm;
            if (conv)
                break;
            if (it >= maxit) {
                status = OMP_NOT_CONVERGED;
                break;
            }
        }
        double beta = 0.0, alpha;
        if (it > 0) {
            beta = gamma / gamma_old;
            alpha = gamma / (delta - beta * gamma / alpha_old);
        } else {
            alpha = gamma / delta;
        }
        if (!(gamma > 0.0) || !isfinite(alpha) || !isfinite(beta) || !(alpha > 0.0)) {
            status = OMP_BREAKDOWN;
            break;
        }
        gamma_old = gamma;
        alpha_old = alpha;
        double g = 0.0, dl = 0.0, nu = 0.0, nr = 0.0;
        /* the merged loop: every vector read once and written once */
#pragma omp parallel for schedule(static) reduction(+ : g, dl, nu, nr)
        for (int i = 0; i < n; ++i) {
            const double zi = nv[i] + beta * z[i];
            const double qi = m[i] + beta * q[i];
            const double si = w[i] + beta * s[i];
            const double pi = u[i] + beta * p[i];
            x[i] = x[i] + alpha * pi;
            const double ri = r[i] - alpha * si;
            const double ui = u[i] - alpha * qi;
            const double wi = w[i] - alpha * zi;
            z[i] = zi;
            q[i] = qi;
            s[i] = si;
            p[i] = pi;
            r[i] = ri;
            u[i] = ui;
            w[i] = wi;
            m[i] = dinv[i] * wi;
            g += ri * ui;
            dl += wi * ui;
            nu += ui * ui;
            nr += ri * ri;
        }
        gamma = g;
        delta = dl;
        uu = nu;
        rr = nr;
        spmv(n, rp, ci, val, m, nv);
        ++it;
    }
    *iters_out = it;
    free(buf);
    return status;
}

/* The number of threads an OpenMP parallel region gets by default. */
int omp_default_threads(void) { return omp_get_max_threads(); }
