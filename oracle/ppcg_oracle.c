/*
 * ppcg_oracle.c -- plain, slow, sequential FP64 reference for the PPCG solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * What it computes (Tiwari & Vadhiyar, "Efficient executions of Pipelined
 * Conjugate Gradient Method on Heterogeneous Architectures"):
 *   - ora_spmv     : y = A x for A in CSR (Section V-A: CSR is the format used),
 *                    each row summed left to right in stored column order.
 *   - ora_jacobi   : the Jacobi preconditioner M = diag(A) (Section V-A),
 *                    stored as dinv_i = 1 / a_ii and applied as dinv (.) v.
 *   - ora_dot      : FP64 sum of products, left to right (default) or with
 *                    Neumaier's compensated summation (ora_set_dot_mode).
 *   - ora_pcg      : Algorithm 1 (PCG, Section III-A).
 *   - ora_pipecg   : Algorithm 2 (PIPECG, Section III-B), with the squared
 *                    residual norm rho = (r, r) computed beside gamma, delta
 *                    and (u, u) for the relative-residual stopping mode.
 *
 * Every product and every sum is rounded separately: the file is compiled
 * with -ffp-contract=off and without any reassociating optimisation.
 *
 * Readings of the paper used here (the paper is silent on them):
 *   - The convergence test sits at the top of the loop, before alpha and
 *     beta (Section IV-C: the residual norm is checked, then alpha and beta
 *     are computed).  "iters" counts x-updates; a converged initial guess
 *     gives 0 iterations.
 *   - Two stopping modes: ORA_STOP_ABS stops when sqrt((u,u)) < tol, the
 *     absolute preconditioned-residual test of the paper's experiments
 *     (Section VI); ORA_STOP_REL stops when sqrt((r,r)) <= tol * ||b||.
 *   - fixed_iters > 0 runs exactly that many iterations and ignores tol; it
 *     stops early only when gamma is exactly 0 (exact solution reached) or on
 *     breakdown.
 *   - Breakdown: gamma <= 0, the alpha denominator <= 0 (for PCG: delta <= 0),
 *     or a non-finite alpha or beta.
 *   - In ORA_STOP_REL mode, when the recurrence reports convergence, the true
 *     residual ||b - A x|| / ||b|| is computed; if it exceeds tol the method is
 *     restarted from the current x (its initialisation steps rerun), at most
 *     max_restarts times, after which the status is ORA_STAGNATED.
 *   - A breakdown after the first iteration of a start (rounding has degraded
 *     the recurrences, as happens to pipelined CG near its attainable
 *     accuracy) restarts the method from the current x in the same way, when
 *     not in fixed-iteration mode and restarts remain; a breakdown at the
 *     first iteration of a start is reported as ORA_BREAKDOWN.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_OK = 0, ORA_NOT_CONVERGED = 1, ORA_BREAKDOWN = 2, ORA_STAGNATED = 3, ORA_BAD_INPUT = -1 };
enum { ORA_STOP_REL = 0, ORA_STOP_ABS = 1 };

typedef struct {
    int iters;
    int restarts;
    int status;
    int pad;
    double rel_true;     /* ||b - A x||_2 / ||b||_2 at exit (||b - A x|| if b == 0) */
    double rel_recur;    /* sqrt((r,r)) / ||b|| of the recurrence residual at exit */
    double precond_norm; /* sqrt((u,u)) at exit */
    double bnorm;        /* ||b||_2 */
} ora_info;

/* y = A x, every row summed in stored order. */
void ora_spmv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            double prod = v[k] * x[ci[k]];
            acc = acc + prod;
        }
        y[i] = acc;
    }
}

/* How ora_dot sums its products: ORA_DOT_SEQ (the default) left to right;
 * ORA_DOT_COMP with Neumaier's compensated summation, which keeps the
 * rounding error of every addition in a second accumulator.  The paper
 * leaves the order of the dot products to its BLAS library, so both are
 * admissible roundings of the same definition; comparing the iterates of the
 * two measures how far any reordering of the sums moves them. */
enum { ORA_DOT_SEQ = 0, ORA_DOT_COMP = 1 };
static int g_dot_mode = ORA_DOT_SEQ;

void ora_set_dot_mode(int mode) { g_dot_mode = mode == ORA_DOT_COMP ? ORA_DOT_COMP : ORA_DOT_SEQ; }

double ora_dot(int n, const double *a, const double *b)
{
    double acc = 0.0;
    if (g_dot_mode == ORA_DOT_COMP) {
        double comp = 0.0; /* sum of the rounding errors of the additions */
        for (int i = 0; i < n; ++i) {
            double prod = a[i] * b[i];
            double t = acc + prod;
            if (fabs(acc) >= fabs(prod))
                comp = comp + ((acc - t) + prod);
            else
                comp = comp + ((prod - t) + acc);
            acc = t;
        }
        return acc + comp;
    }
    for (int i = 0; i < n; ++i) {
        double prod = a[i] * b[i];
        acc = acc + prod;
    }
    return acc;
}

/* dinv_i = 1 / a_ii.  Returns 0, or -1 if a diagonal is missing or not > 0. */
int ora_jacobi(int n, const int *rp, const int *ci, const double *v, double *dinv)
{
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        int found = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] == i) {
                d = v[k];
                found = 1;
            }
        }
        if (!found || !(d > 0.0))
            return -1;
        dinv[i] = 1.0 / d;
    }
    return 0;
}

/* ||b - A x|| / ||b|| (plain ||b - A x|| when b == 0). */
double ora_true_relres(int n, const int *rp, const int *ci, const double *v, const double *b,
                       const double *x)
{
    double *ax = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    ora_spmv(n, rp, ci, v, x, ax);
    double rr = 0.0, bb = 0.0;
    for (int i = 0; i < n; ++i) {
        double d = b[i] - ax[i];
        rr = rr + d * d;
        bb = bb + b[i] * b[i];
    }
    free(ax);
    return bb > 0.0 ? sqrt(rr) / sqrt(bb) : sqrt(rr);
}

static int converged(int stop, double tol, double bnorm, double uu, double rr)
{
    if (stop == ORA_STOP_ABS)
        return sqrt(uu) < tol;
    return sqrt(rr) <= tol * bnorm;
}

static double *vec(int n)
{
    return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
}

/*
 * Algorithm 1 (PCG).
 *   r0 = b - A x0;  u0 = M^-1 r0;  gamma0 = (u0, r0);  norm0 = sqrt((u0, u0))
 *   loop: beta = gamma_i / gamma_{i-1} (0 at i = 0);  p = u + beta p;  s = A p;
 *         delta = (s, p);  alpha = gamma / delta;  x += alpha p;  r -= alpha s;
 *         u = M^-1 r;  gamma = (u, r);  norm = sqrt((u, u)).
 * hist (may be NULL) receives the stopping quantity at each loop top,
 * at most hist_len entries.
 */
int ora_pcg(int n, const int *rp, const int *ci, const double *v, const double *b, const double *x0,
            double *x, double tol, int maxit, int fixed_iters, int stop, int max_restarts, ora_info *info,
            double *hist, int hist_len)
{
    memset(info, 0, sizeof(*info));
    double *dinv = vec(n), *r = vec(n), *u = vec(n), *p = vec(n), *s = vec(n);
    if (ora_jacobi(n, rp, ci, v, dinv) != 0) {
        info->status = ORA_BAD_INPUT;
        free(dinv); free(r); free(u); free(p); free(s);
        return ORA_BAD_INPUT;
    }
    for (int i = 0; i < n; ++i)
        x[i] = x0 ? x0[i] : 0.0;
    const double bnorm = sqrt(ora_dot(n, b, b));
    int it = 0, restarts = 0, status = ORA_OK;
    double gamma = 0.0, uu = 0.0, rr = 0.0;
    for (;;) {
        /* Algorithm 1 initialisation: r0, u0, gamma0, norm0 */
        ora_spmv(n, rp, ci, v, x, r);
        for (int i = 0; i < n; ++i) {
            r[i] = b[i] - r[i];
            u[i] = dinv[i] * r[i];
            p[i] = 0.0;
        }
        gamma = ora_dot(n, u, r);
        uu = ora_dot(n, u, u);
        rr = ora_dot(n, r, r);
        double gamma_prev = 0.0;
        int i; /* iteration index within the current start */
        for (i = 0;; ++i) {
            double q = stop == ORA_STOP_ABS ? sqrt(uu) : sqrt(rr);
            if (hist && it < hist_len)
                hist[it] = q;
            if (fixed_iters > 0) {
                if (it >= fixed_iters || gamma == 0.0) { status = ORA_OK; break; }
            } else {
                if (converged(stop, tol, bnorm, uu, rr)) { status = ORA_OK; break; }
                if (it >= maxit) { status = ORA_NOT_CONVERGED; break; }
            }
            double beta = i > 0 ? gamma / gamma_prev : 0.0;      /* beta */
            for (int k = 0; k < n; ++k)                           /* search direction */
                p[k] = u[k] + beta * p[k];
            ora_spmv(n, rp, ci, v, p, s);
            double delta = ora_dot(n, s, p);
            double alpha = gamma / delta;
            if (!(gamma > 0.0) || !(delta > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
                status = ORA_BREAKDOWN;
                break;
            }
            for (int k = 0; k < n; ++k) {
                x[k] = x[k] + alpha * p[k];
                r[k] = r[k] - alpha * s[k];
                u[k] = dinv[k] * r[k];
            }
            gamma_prev = gamma;
            gamma = ora_dot(n, u, r);
            uu = ora_dot(n, u, u);
            rr = ora_dot(n, r, r);
            ++it;
        }
        if (status == ORA_BREAKDOWN && fixed_iters <= 0 && i > 0 && restarts < max_restarts &&
            it < maxit) {
            ++restarts;
            continue;
        }
        if (status == ORA_OK && fixed_iters <= 0 && stop == ORA_STOP_REL) {
            double rel = ora_true_relres(n, rp, ci, v, b, x);
            if (rel > tol) {
                if (restarts < max_restarts && it < maxit) {
                    ++restarts;
                    continue;
                }
                status = ORA_STAGNATED;
            }
        }
        break;
    }
    info->iters = it;
    info->restarts = restarts;
    info->status = status;
    info->bnorm = bnorm;
    info->rel_true = ora_true_relres(n, rp, ci, v, b, x);
    info->rel_recur = bnorm > 0.0 ? sqrt(rr) / bnorm : sqrt(rr);
    info->precond_norm = sqrt(uu);
    free(dinv); free(r); free(u); free(p); free(s);
    return status;
}

/*
 * Algorithm 2 (PIPECG).
 *   init : r0 = b - A x0;  u0 = M^-1 r0;  w0 = A u0;
 *          gamma0 = (r0, u0);  delta = (w0, u0);  norm0 = sqrt((u0, u0));
 *          m0 = M^-1 w0;  n0 = A m0
 *   loop : beta = gamma_i / gamma_{i-1},
 *          alpha = gamma_i / (delta - beta gamma_i / alpha_{i-1})
 *          (beta = 0, alpha = gamma_0 / delta at i = 0);
 *          z = n + beta z;  q = m + beta q;  s = w + beta s;  p = u + beta p;
 *          x += alpha p;  r -= alpha s;  u -= alpha q;  w -= alpha z;
 *          gamma = (r, u);  delta = (w, u);  norm = sqrt((u, u));
 *          m = M^-1 w;  n = A m.
 * state (may be NULL) receives, at exit, the ten vectors
 * x r u w m n z q s p (10 n doubles) followed by the scalars
 * gamma, delta, (u,u), (r,r), alpha_{i-1}, gamma_{i-1}, beta_{i-1}.
 */
int ora_pipecg(int n, const int *rp, const int *ci, const double *v, const double *b, const double *x0,
               double *x, double tol, int maxit, int fixed_iters, int stop, int max_restarts, ora_info *info,
               double *hist, int hist_len, double *state)
{
    memset(info, 0, sizeof(*info));
    double *dinv = vec(n), *r = vec(n), *u = vec(n), *w = vec(n), *m = vec(n), *nv = vec(n);
    double *z = vec(n), *q = vec(n), *s = vec(n), *p = vec(n);
    int status = ORA_OK;
    if (ora_jacobi(n, rp, ci, v, dinv) != 0) {
        info->status = ORA_BAD_INPUT;
        status = ORA_BAD_INPUT;
        goto out;
    }
    for (int i = 0; i < n; ++i)
        x[i] = x0 ? x0[i] : 0.0;
    const double bnorm = sqrt(ora_dot(n, b, b));
    int it = 0, restarts = 0;
    double gamma = 0.0, delta = 0.0, uu = 0.0, rr = 0.0;
    double alpha_prev = 0.0, gamma_prev = 0.0, beta = 0.0;
    for (;;) {
        /* Algorithm 2 initialisation: r0, u0, w0 */
        ora_spmv(n, rp, ci, v, x, r);
        for (int i = 0; i < n; ++i) {
            r[i] = b[i] - r[i];
            u[i] = dinv[i] * r[i];
            z[i] = q[i] = s[i] = p[i] = 0.0;
        }
        ora_spmv(n, rp, ci, v, u, w);
        /* gamma0, delta, norm0 (and rho0) */
        gamma = ora_dot(n, r, u);
        delta = ora_dot(n, w, u);
        uu = ora_dot(n, u, u);
        rr = ora_dot(n, r, r);
        /* m0, n0 */
        for (int i = 0; i < n; ++i)
            m[i] = dinv[i] * w[i];
        ora_spmv(n, rp, ci, v, m, nv);
        int i; /* iteration index within the current start */
        for (i = 0;; ++i) {
            double qn = stop == ORA_STOP_ABS ? sqrt(uu) : sqrt(rr);
            if (hist && it < hist_len)
                hist[it] = qn;
            if (fixed_iters > 0) {
                if (it >= fixed_iters || gamma == 0.0) { status = ORA_OK; break; }
            } else {
                if (converged(stop, tol, bnorm, uu, rr)) { status = ORA_OK; break; }
                if (it >= maxit) { status = ORA_NOT_CONVERGED; break; }
            }
            double alpha, denom;
            if (i > 0) {                                           /* i > 0 */
                beta = gamma / gamma_prev;
                denom = delta - beta * gamma / alpha_prev;
            } else {                                               /* i == 0 */
                beta = 0.0;
                denom = delta;
            }
            alpha = gamma / denom;
            if (!(gamma > 0.0) || !(denom > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
                status = ORA_BREAKDOWN;
                break;
            }
            for (int k = 0; k < n; ++k) {
                z[k] = nv[k] + beta * z[k];
                q[k] = m[k] + beta * q[k];
                s[k] = w[k] + beta * s[k];
                p[k] = u[k] + beta * p[k];
                x[k] = x[k] + alpha * p[k];
                r[k] = r[k] - alpha * s[k];
                u[k] = u[k] - alpha * q[k];
                w[k] = w[k] - alpha * z[k];
            }
            gamma_prev = gamma;
            alpha_prev = alpha;
            gamma = ora_dot(n, r, u);
            delta = ora_dot(n, w, u);
            uu = ora_dot(n, u, u);
            rr = ora_dot(n, r, r);
            for (int k = 0; k < n; ++k)
                m[k] = dinv[k] * w[k];
            ora_spmv(n, rp, ci, v, m, nv);
            ++it;
        }
        if (status == ORA_BREAKDOWN && fixed_iters <= 0 && i > 0 && restarts < max_restarts &&
            it < maxit) {
            ++restarts;
            continue;
        }
        if (status == ORA_OK && fixed_iters <= 0 && stop == ORA_STOP_REL) {
            double rel = ora_true_relres(n, rp, ci, v, b, x);
            if (rel > tol) {
                if (restarts < max_restarts && it < maxit) {
                    ++restarts;
                    continue;
                }
                status = ORA_STAGNATED;
            }
        }
        break;
    }
    info->iters = it;
    info->restarts = restarts;
    info->status = status;
    info->bnorm = bnorm;
    info->rel_true = ora_true_relres(n, rp, ci, v, b, x);
    info->rel_recur = bnorm > 0.0 ? sqrt(rr) / bnorm : sqrt(rr);
    info->precond_norm = sqrt(uu);
    if (state) {
        double *vs[10] = {x, r, u, w, m, nv, z, q, s, p};
        for (int j = 0; j < 10; ++j)
            memcpy(state + (size_t)j * n, vs[j], sizeof(double) * (size_t)n);
        double *sc = state + (size_t)10 * n;
        sc[0] = gamma; sc[1] = delta; sc[2] = uu; sc[3] = rr;
        sc[4] = alpha_prev; sc[5] = gamma_prev; sc[6] = beta;
    }
out:
    free(dinv); free(r); free(u); free(w); free(m); free(nv);
    free(z); free(q); free(s); free(p);
    return status;
}
