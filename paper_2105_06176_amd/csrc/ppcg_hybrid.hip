// ppcg_hybrid.hip -- Algorithm 2 run by host cores and the GPU together, in
// the three execution schemes of Tiwari & Vadhiyar (Section IV).  Most of this
// file is the data-parallel Hybrid-PIPECG-3 (Section IV-C); the task-parallel
// Hybrid-PIPECG-1 and -2 (Sections IV-A, IV-B) are solve_task below.
//
// Hybrid-PIPECG-3.
// Setup: both sides time five SpMVs over all of A; the performance model
// splits the rows (ppcg_split_rows): rows [0, ncpu) go to the host, the rest
// to the GPU.  Each side's entries are split into part 1 (columns it owns)
// and part 2 (columns the other side owns), the 2-D decomposition.
//
// One iteration follows the paper's execution flow.  With alpha and beta
// known on the host:
//   1. the m entries each side needs from the other start moving (GPU -> host
//      into pinned memory, host -> GPU into the GPU's halo buffer);
//   2. both sides update the vectors that do not depend on n:
//      q = m + beta q, s = w + beta s, p = u + beta p, x += alpha p,
//      r -= alpha s, u -= alpha q, with partial sums of (r,u), (u,u), (r,r);
//   3. SpMV part 1, n = A_local m;
//   4. once the copy has arrived, SpMV part 2, n += A_remote m_halo;
//   5. z = n + beta z, w -= alpha z, m = M^-1 w, partial sum of (w,u);
//   6. the host adds the two sides' partial sums (host first, then GPU) and
//      runs the stopping test and the scalar recurrences of Algorithm 2.
// This is Algorithm 2 with n = A m computed at the start of the iteration
// that uses it rather than at the end of the previous one.
//
// Host work runs on a small pool of threads with static row ranges; every
// sum the host forms is taken in a fixed order (rows in order per thread,
// threads in order), so results are reproducible.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ppcg_engine.hpp"
#include "ppcg_shard_internal.hpp"

using namespace ppcg;

namespace {

constexpr int kH3Threads = 256;  // GPU update kernels: one row per thread
constexpr int kH3RedThreads = 1024;

// ------------------------------------------------------------------ GPU side

// Step 2 on the GPU rows, with per-block partial sums of (r,u), (u,u), (r,r).
__global__ __launch_bounds__(kH3Threads) void k_h3_update1(int n, double alpha, double beta,
                                                           const double *__restrict__ m, double *__restrict__ q,
                                                           const double *__restrict__ w, double *__restrict__ s,
                                                           double *__restrict__ u, double *__restrict__ p,
                                                           double *__restrict__ x, double *__restrict__ r,
                                                           double *__restrict__ part)
{
    __shared__ double lds[kH3Threads / 64 * 3];
    const int i = blockIdx.x * kH3Threads + threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (i < n) {
        const double qi = m[i] + beta * q[i];
        const double si = w[i] + beta * s[i];
        const double pi = u[i] + beta * p[i];
        const double xi = x[i] + alpha * pi;
        const double ri = r[i] - alpha * si;
        const double ui = u[i] - alpha * qi;
        q[i] = qi;
        s[i] = si;
        p[i] = pi;
        x[i] = xi;
        r[i] = ri;
        u[i] = ui;
        a0 = ri * ui;
        a1 = ui * ui;
        a2 = ri * ri;
    }
    // fixed-order block reduction
    for (int off = 32; off >= 1; off >>= 1) {
        a0 = a0 + __shfl_xor(a0, off, 64);
        a1 = a1 + __shfl_xor(a1, off, 64);
        a2 = a2 + __shfl_xor(a2, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        lds[wv * 3 + 0] = a0;
        lds[wv * 3 + 1] = a1;
        lds[wv * 3 + 2] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b0 = lds[0], b1 = lds[1], b2 = lds[2];
        for (int k = 1; k < kH3Threads / 64; ++k) {
            b0 = b0 + lds[k * 3 + 0];
            b1 = b1 + lds[k * 3 + 1];
            b2 = b2 + lds[k * 3 + 2];
        }
        part[(size_t)blockIdx.x * 4 + 0] = b0;
        part[(size_t)blockIdx.x * 4 + 1] = b1;
        part[(size_t)blockIdx.x * 4 + 2] = b2;
    }
}

// Step 5 on the GPU rows, with per-block partial sums of (w,u).
__global__ __launch_bounds__(kH3Threads) void k_h3_update2(int n, double alpha, double beta,
                                                           const double *__restrict__ nv, double *__restrict__ z,
                                                           double *__restrict__ w, double *__restrict__ m,
                                                           const double *__restrict__ dinv,
                                                           const double *__restrict__ u, double *__restrict__ part)
{
    __shared__ double lds[kH3Threads / 64];
    const int i = blockIdx.x * kH3Threads + threadIdx.x;
    double a = 0.0;
    if (i < n) {
        const double zi = nv[i] + beta * z[i];
        const double wi = w[i] - alpha * zi;
        z[i] = zi;
        w[i] = wi;
        m[i] = dinv[i] * wi;
        a = wi * u[i];
    }
    for (int off = 32; off >= 1; off >>= 1)
        a = a + __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0)
        lds[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = lds[0];
        for (int k = 1; k < kH3Threads / 64; ++k)
            b = b + lds[k];
        part[(size_t)blockIdx.x * 4 + 3] = b;
    }
}

// Initialisation on the GPU rows: r = b - y (y = A x0, or r = b when x0 = 0 and
// y is NULL), u = M^-1 r; z = q = s = p = 0.
__global__ void k_h3_init1(int n, const double *__restrict__ b, const double *__restrict__ y,
                           const double *__restrict__ dinv, double *__restrict__ r, double *__restrict__ u,
                           double *__restrict__ z, double *__restrict__ q, double *__restrict__ s,
                           double *__restrict__ p)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double ri = y ? b[i] - y[i] : b[i];
        r[i] = ri;
        u[i] = dinv[i] * ri;
        z[i] = q[i] = s[i] = p[i] = 0.0;
    }
}

// Initialisation, after w = A u: m = M^-1 w and the four partial sums.
__global__ __launch_bounds__(kH3Threads) void k_h3_init2(int n, const double *__restrict__ r,
                                                         const double *__restrict__ u, const double *__restrict__ w,
                                                         const double *__restrict__ dinv, double *__restrict__ m,
                                                         double *__restrict__ part)
{
    __shared__ double lds[kH3Threads / 64 * 4];
    const int i = blockIdx.x * kH3Threads + threadIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        m[i] = dinv[i] * w[i];
        a[0] = r[i] * u[i];
        a[1] = u[i] * u[i];
        a[2] = r[i] * r[i];
        a[3] = w[i] * u[i];
    }
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off >= 1; off >>= 1)
            a[k] = a[k] + __shfl_xor(a[k], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k)
            lds[(threadIdx.x >> 6) * 4 + k] = a[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) {
            double t = lds[k];
            for (int v = 1; v < kH3Threads / 64; ++v)
                t = t + lds[v * 4 + k];
            part[(size_t)blockIdx.x * 4 + k] = t;
        }
}

// One workgroup: the four block partials summed in block order (each thread
// its blocks in order, then the workgroup tree) into out[0..3].
__global__ __launch_bounds__(kH3RedThreads) void k_h3_reduce(int nblocks, const double *__restrict__ part,
                                                             double *__restrict__ out)
{
    __shared__ double lds[kH3RedThreads / 64 * 4];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int blk = threadIdx.x; blk < nblocks; blk += kH3RedThreads)
        for (int k = 0; k < 4; ++k)
            a[k] = a[k] + part[(size_t)blk * 4 + k];
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off >= 1; off >>= 1)
            a[k] = a[k] + __shfl_xor(a[k], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k)
            lds[(threadIdx.x >> 6) * 4 + k] = a[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) {
            double t = lds[k];
            for (int v = 1; v < kH3RedThreads / 64; ++v)
                t = t + lds[v * 4 + k];
            out[k] = t;
        }
}

// Compact the GPU-owned entries the host needs: out[k] = v[cols[k] - base].
__global__ void k_h3_pack(int h, const int *__restrict__ cols, int base, const double *__restrict__ v,
                          double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < h)
        out[k] = v[cols[k] - base];
}

// ------------------------------------------------------------------ host side

// A fixed set of worker threads running one function over thread ids; the
// caller runs id 0 itself.  Idle workers spin briefly (with yields) for the
// next generation, then sleep on a condition variable.
class HostPool {
  public:
    explicit HostPool(int t) : nt_(std::max(1, t))
    {
        for (int k = 1; k < nt_; ++k)
            th_.emplace_back([this]() { worker(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true);
            gen_.fetch_add(1);
        }
        cv_.notify_all();
        for (auto &t : th_)
            t.join();
    }
    int size() const { return nt_; }
    void run(const std::function<void(int)> &f)
    {
        job_ = &f;
        pending_.store(nt_ - 1);
        next_id_.store(1);
        {
            std::lock_guard<std::mutex> lk(mu_);
            gen_.fetch_add(1, std::memory_order_release);
        }
        cv_.notify_all();
        f(0);
        while (pending_.load(std::memory_order_acquire) != 0)
            std::this_thread::yield();
        job_ = nullptr;
    }

  private:
    void worker()
    {
        unsigned seen = 0;
        for (;;) {
            unsigned g;
            int spins = 0;
            while ((g = gen_.load(std::memory_order_acquire)) == seen) {
                if (++spins < 4096) {
                    std::this_thread::yield();
                    continue;
                }
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&]() { return gen_.load(std::memory_order_acquire) != seen; });
            }
            seen = g;
            if (stop_.load())
                return;
            // thread ids 1 .. nt-1, handed out per generation
            const int id = next_id_.fetch_add(1);
            (*job_)(id);
            pending_.fetch_sub(1, std::memory_order_acq_rel);
        }
    }
    int nt_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::atomic<unsigned> gen_{0};
    std::atomic<int> pending_{0}, next_id_{1};
    std::atomic<bool> stop_{false};
    const std::function<void(int)> *job_ = nullptr;
};

struct HostCsr {
    std::vector<int> rp, ci;
    std::vector<double> val;
};

}  // namespace

struct ppcg_hybrid {
    int device = 0;
    int scheme = PPCG_HYBRID_3;
    hipStream_t stream = nullptr;
    ppcg_options opt{};
    int n = 0, ncpu = 0, ngpu = 0;
    double t_cpu = 0.0, t_gpu = 0.0;  // seconds per full SpMV (performance model)
    std::unique_ptr<HostPool> pool;
    std::vector<int> row_lo;          // per host thread: first row (size threads + 1)
    // host rows [0, ncpu): part 1 (local columns) and part 2 (columns of the
    // GPU's rows, numbered by position in hcols)
    HostCsr h1, h2;
    std::vector<int> hcols;           // GPU-owned columns the host reads, ascending
    std::vector<double> dinv_h;
    std::vector<double> x, r, u, w, m, nv, z, q, s, p, bh;
    // GPU rows [ncpu, n)
    ppcg_shard *gs = nullptr;         // part 1 / part 2 SpMV, halo = host-owned columns
    DevArena arena;
    double *dx = nullptr, *dr = nullptr, *du = nullptr, *dw = nullptr, *dm = nullptr, *dn = nullptr;
    double *dz = nullptr, *dq = nullptr, *ds = nullptr, *dp = nullptr, *ddinv = nullptr, *db = nullptr;
    double *dy = nullptr, *dpart = nullptr, *dred = nullptr, *dhalo = nullptr, *dpack = nullptr;
    int *dhcols = nullptr;
    int nblocks = 0;
    // pinned staging
    double *pin_to_host = nullptr;    // GPU-owned entries for the host [hcols.size()]
    double *pin_to_dev = nullptr;     // host-owned entries for the GPU [gs->halo]
    double *pin_red = nullptr;        // GPU scalars [4]
    hipEvent_t ev_halo = nullptr;
    // Hybrid-1 / -2 (every row on the GPU): the copy stream, its events, the
    // pinned copies (Hybrid-1: w, r, u; Hybrid-2: n) and Hybrid-2's host
    // vectors
    hipStream_t cstream = nullptr;
    hipEvent_t ev_upd = nullptr, ev_copy = nullptr;
    double *pin_vec = nullptr;
    std::vector<int> full_lo;         // per host thread: first row of [0, n)
};

namespace {

// Host SpMV over rows [lo, hi) of the host part: y = A1 v_local + A2 v_halo.
void host_spmv_rows(const ppcg_hybrid *hy, int lo, int hi, const double *vl, const double *vh, double *y,
                    bool part1, bool part2)
{
    for (int i = lo; i < hi; ++i) {
        if (part1) {
            double a = 0.0;
            for (int k = hy->h1.rp[i]; k < hy->h1.rp[i + 1]; ++k)
                a = a + hy->h1.val[k] * vl[hy->h1.ci[k]];
            y[i] = a;
        }
        if (part2 && hy->h2.rp[i + 1] > hy->h2.rp[i]) {
            double a = 0.0;
            for (int k = hy->h2.rp[i]; k < hy->h2.rp[i + 1]; ++k)
                a = a + hy->h2.val[k] * vh[hy->h2.ci[k]];
            y[i] = y[i] + a;
        }
    }
}

// Pack the host-owned entries the GPU needs into pinned memory (in the
// order of the GPU shard's halo list).
void host_pack(ppcg_hybrid *hy, const double *v)
{
    const std::vector<int> &hc = hy->gs->halo_cols;
    for (size_t k = 0; k < hc.size(); ++k)
        hy->pin_to_dev[k] = v[hc[k]];
}

// y = A v over all rows, with v split as (host rows: vh_rows, GPU rows:
// dv), result in (host: yh, GPU: dy).  Used by the initialisation and the
// final true residual.  Synchronous.
ppcg_status hybrid_spmv(ppcg_hybrid *hy, const double *vh_rows, const double *dv, double *yh, double *dy)
{
    hipStream_t st = hy->stream;
    const int hc = (int)hy->hcols.size();
    if (hy->ngpu > 0) {
        if (hy->gs->halo > 0) {
            host_pack(hy, vh_rows);
            PPCG_HIP(hipMemcpyAsync(hy->dhalo, hy->pin_to_dev, sizeof(double) * hy->gs->halo,
                                    hipMemcpyHostToDevice, st));
        }
        if (hc > 0) {
            k_h3_pack<<<(hc + 255) / 256, 256, 0, st>>>(hc, hy->dhcols, hy->ncpu, dv, hy->dpack);
            PPCG_HIP(hipMemcpyAsync(hy->pin_to_host, hy->dpack, sizeof(double) * hc, hipMemcpyDeviceToHost, st));
        }
        PPCG_TRY(shard_launch(hy->gs, 1, dv, hy->dhalo, dy, nullptr, nullptr));
        PPCG_TRY(shard_launch(hy->gs, 2, dv, hy->dhalo, dy, nullptr, nullptr));
        PPCG_HIP(hipStreamSynchronize(st));
    }
    hy->pool->run([&](int t) {
        host_spmv_rows(hy, hy->row_lo[t], hy->row_lo[t + 1], vh_rows, hy->pin_to_host, yh, true, true);
    });
    return PPCG_OK;
}

double host_dot_rows(const ppcg_hybrid *hy, const std::vector<double> &a, const std::vector<double> &b,
                     std::vector<double> &per_thread)
{
    hy->pool->run([&](int t) {
        double acc = 0.0;
        for (int i = hy->row_lo[t]; i < hy->row_lo[t + 1]; ++i)
            acc = acc + a[i] * b[i];
        per_thread[t] = acc;
    });
    double s = 0.0;
    for (int t = 0; t < hy->pool->size(); ++t)
        s = s + per_thread[t];
    return s;
}

// ||b - A x|| over all rows: host rows from hy->x and hy->bh, GPU rows from
// hy->dx and hy->db (synchronous).
ppcg_status hybrid_resid_norm(ppcg_hybrid *hy, const double *xh_rows, double *t2_out)
{
    const int nc = hy->ncpu, ng = hy->ngpu;
    std::vector<double> yh(nc);
    PPCG_TRY(hybrid_spmv(hy, xh_rows, hy->dx, yh.data(), hy->dy));
    double t2 = 0.0;
    for (int k = 0; k < nc; ++k) {
        const double d = hy->bh[k] - yh[k];
        t2 = t2 + d * d;
    }
    std::vector<double> yg(ng), bg(ng);
    if (ng > 0) {
        PPCG_HIP(hipMemcpy(yg.data(), hy->dy, sizeof(double) * ng, hipMemcpyDeviceToHost));
        PPCG_HIP(hipMemcpy(bg.data(), hy->db, sizeof(double) * ng, hipMemcpyDeviceToHost));
    }
    for (int k = 0; k < ng; ++k) {
        const double d = bg[k] - yg[k];
        t2 = t2 + d * d;
    }
    *t2_out = t2;
    return PPCG_OK;
}

// Hybrid-PIPECG-1 and -2 (Sections IV-A, IV-B): every row on the GPU.  The GPU
// stream runs, per iteration, the updates of q, s, p, x, r, u
// (k_h3_update1), of z, w, m with the n of the previous SpMV (k_h3_update2),
// then the SpMV n = A m for the next iteration.  The copy stream moves, after
// the updates, w, r, u (Hybrid-1) or, after the SpMV, n (Hybrid-2) to pinned
// host memory; the host computes the dot products and alpha and beta.
// Hybrid-2's host repeats the updates of q, s, r, u (and gamma, the norms)
// while n is in flight, then z, w, m (and delta) once it has arrived; its
// copies are bitwise the GPU's (same operations, same order).  Two n buffers
// alternate so that the copy of one overlaps the SpMV writing the other: the
// host waits for a copy before it lets the GPU run the iteration after.
ppcg_status solve_task(ppcg_hybrid *hy, const double *b, const double *x0, double *x, ppcg_info *info)
{
    const auto t_begin = std::chrono::steady_clock::now();
    const int n = hy->n;
    const int T = hy->pool->size();
    const std::vector<int> &lo = hy->full_lo;
    hipStream_t st = hy->stream, cs = hy->cstream;
    const ppcg_options &o = hy->opt;
    const int g1 = (n + kH3Threads - 1) / kH3Threads;
    const bool h2 = hy->scheme == PPCG_HYBRID_2;
    double *nbuf[2] = {hy->dn, hy->dy};  // dy is free during the iterations
    double *pin_w = hy->pin_vec, *pin_r = hy->pin_vec + (h2 ? 0 : n), *pin_u = hy->pin_vec + (h2 ? 0 : 2 * (size_t)n);
    double *pin_n = hy->pin_vec;
    std::vector<double> pt(T), pt4(4 * T);
    PPCG_HIP(hipMemcpyAsync(hy->db, b, sizeof(double) * n, hipMemcpyHostToDevice, st));
    if (x0)
        PPCG_HIP(hipMemcpyAsync(hy->dx, x0, sizeof(double) * n, hipMemcpyHostToDevice, st));
    else
        PPCG_HIP(hipMemsetAsync(hy->dx, 0, sizeof(double) * n, st));
    hy->pool->run([&](int t) {
        double a = 0.0;
        for (int i = lo[t]; i < lo[t + 1]; ++i)
            a = a + b[i] * b[i];
        pt[t] = a;
    });
    double bb = 0.0;
    for (int t = 0; t < T; ++t)
        bb = bb + pt[t];
    const double bnorm = std::sqrt(bb);
    // gamma = (r,u), (u,u), (r,r), delta = (w,u) over all rows, threads in order
    auto host_dots = [&](const double *r, const double *u, const double *w, double *g) {
        hy->pool->run([&](int t) {
            double a[4] = {0, 0, 0, 0};
            for (int i = lo[t]; i < lo[t + 1]; ++i) {
                a[0] = a[0] + r[i] * u[i];
                a[1] = a[1] + u[i] * u[i];
                a[2] = a[2] + r[i] * r[i];
                a[3] = a[3] + w[i] * u[i];
            }
            for (int k = 0; k < 4; ++k)
                pt4[4 * t + k] = a[k];
        });
        for (int k = 0; k < 4; ++k) {
            g[k] = 0.0;
            for (int t = 0; t < T; ++t)
                g[k] = g[k] + pt4[4 * t + k];
        }
    };
    int it = 0, restarts = 0, status = PPCG_OK;
    double gamma = 0, delta = 0, uu = 0, rr = 0, alpha_prev = 0, gamma_prev = 0, beta = 0;
    auto converged = [&]() {
        if (o.stop == PPCG_STOP_PRECOND_ABS)
            return std::sqrt(uu) < o.tol;
        return std::sqrt(rr) <= o.tol * bnorm;
    };
    for (;;) {
        // Algorithm 2 initialisation on the GPU; n0 = A m0 into nbuf[0]
        PPCG_TRY(hybrid_spmv(hy, nullptr, hy->dx, nullptr, hy->dy));
        k_h3_init1<<<(n + 255) / 256, 256, 0, st>>>(n, hy->db, hy->dy, hy->ddinv, hy->dr, hy->du, hy->dz, hy->dq,
                                                    hy->ds, hy->dp);
        PPCG_TRY(hybrid_spmv(hy, nullptr, hy->du, nullptr, hy->dw));
        k_h3_init2<<<g1, kH3Threads, 0, st>>>(n, hy->dr, hy->du, hy->dw, hy->ddinv, hy->dm, hy->dpart);
        PPCG_TRY(shard_launch(hy->gs, 1, hy->dm, hy->dhalo, nbuf[0], nullptr, nullptr));
        double g[4];
        if (h2) {
            // the host's copies: r, u, w, m; z = q = s = 0; and n0 in flight
            PPCG_HIP(hipMemcpyAsync(hy->r.data(), hy->dr, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipMemcpyAsync(hy->u.data(), hy->du, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipMemcpyAsync(hy->w.data(), hy->dw, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipMemcpyAsync(hy->m.data(), hy->dm, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipEventRecord(hy->ev_upd, st));
            PPCG_HIP(hipStreamWaitEvent(cs, hy->ev_upd, 0));
            PPCG_HIP(hipMemcpyAsync(pin_n, nbuf[0], sizeof(double) * n, hipMemcpyDeviceToHost, cs));
            PPCG_HIP(hipEventRecord(hy->ev_copy, cs));
            PPCG_HIP(hipStreamSynchronize(st));
            std::fill(hy->z.begin(), hy->z.end(), 0.0);
            std::fill(hy->q.begin(), hy->q.end(), 0.0);
            std::fill(hy->s.begin(), hy->s.end(), 0.0);
            host_dots(hy->r.data(), hy->u.data(), hy->w.data(), g);
        } else {
            PPCG_HIP(hipMemcpyAsync(pin_w, hy->dw, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipMemcpyAsync(pin_r, hy->dr, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipMemcpyAsync(pin_u, hy->du, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipStreamSynchronize(st));
            host_dots(pin_r, pin_u, pin_w, g);
        }
        gamma = g[0];
        uu = g[1];
        rr = g[2];
        delta = g[3];
        int i;
        for (i = 0;; ++i) {
            if (o.fixed_iters > 0) {
                if (it >= o.fixed_iters || gamma == 0.0) {
                    status = PPCG_OK;
                    break;
                }
            } else {
                if (converged()) {
                    status = PPCG_OK;
                    break;
                }
                if (it >= o.max_iter) {
                    status = PPCG_NOT_CONVERGED;
                    break;
                }
            }
            double denom;
            if (i > 0) {
                beta = gamma / gamma_prev;
                denom = delta - beta * gamma / alpha_prev;
            } else {
                beta = 0.0;
                denom = delta;
            }
            const double alpha = gamma / denom;
            if (!(gamma > 0.0) || !(denom > 0.0) || !std::isfinite(alpha) || !std::isfinite(beta)) {
                status = PPCG_BREAKDOWN;
                break;
            }
            double *ncur = nbuf[i & 1], *nnext = nbuf[(i + 1) & 1];
            // GPU: the vector updates of this iteration, then the next n
            k_h3_update1<<<g1, kH3Threads, 0, st>>>(n, alpha, beta, hy->dm, hy->dq, hy->dw, hy->ds, hy->du, hy->dp,
                                                    hy->dx, hy->dr, hy->dpart);
            k_h3_update2<<<g1, kH3Threads, 0, st>>>(n, alpha, beta, ncur, hy->dz, hy->dw, hy->dm, hy->ddinv,
                                                    hy->du, hy->dpart);
            PPCG_HIP(hipGetLastError());
            if (!h2) {
                // Hybrid-1: w, r, u move while the GPU runs the SpMV
                PPCG_HIP(hipEventRecord(hy->ev_upd, st));
                PPCG_HIP(hipStreamWaitEvent(cs, hy->ev_upd, 0));
                PPCG_HIP(hipMemcpyAsync(pin_w, hy->dw, sizeof(double) * n, hipMemcpyDeviceToHost, cs));
                PPCG_HIP(hipMemcpyAsync(pin_r, hy->dr, sizeof(double) * n, hipMemcpyDeviceToHost, cs));
                PPCG_HIP(hipMemcpyAsync(pin_u, hy->du, sizeof(double) * n, hipMemcpyDeviceToHost, cs));
                PPCG_HIP(hipEventRecord(hy->ev_copy, cs));
                PPCG_TRY(shard_launch(hy->gs, 1, hy->dm, hy->dhalo, nnext, nullptr, nullptr));
                PPCG_HIP(hipEventSynchronize(hy->ev_copy));
                host_dots(pin_r, pin_u, pin_w, g);
            } else {
                // Hybrid-2: the host repeats the updates; the copy of this
                // iteration's n (enqueued after the previous SpMV) is waited
                // for only before z, w, m
                PPCG_TRY(shard_launch(hy->gs, 1, hy->dm, hy->dhalo, nnext, nullptr, nullptr));
                hy->pool->run([&](int t) {
                    double a0 = 0, a1 = 0, a2 = 0;
                    for (int k = lo[t]; k < lo[t + 1]; ++k) {
                        hy->q[k] = hy->m[k] + beta * hy->q[k];
                        hy->s[k] = hy->w[k] + beta * hy->s[k];
                        hy->r[k] = hy->r[k] - alpha * hy->s[k];
                        hy->u[k] = hy->u[k] - alpha * hy->q[k];
                        a0 = a0 + hy->r[k] * hy->u[k];
                        a1 = a1 + hy->u[k] * hy->u[k];
                        a2 = a2 + hy->r[k] * hy->r[k];
                    }
                    pt4[4 * t + 0] = a0;
                    pt4[4 * t + 1] = a1;
                    pt4[4 * t + 2] = a2;
                });
                PPCG_HIP(hipEventSynchronize(hy->ev_copy));
                hy->pool->run([&](int t) {
                    double a3 = 0.0;
                    for (int k = lo[t]; k < lo[t + 1]; ++k) {
                        hy->z[k] = pin_n[k] + beta * hy->z[k];
                        hy->w[k] = hy->w[k] - alpha * hy->z[k];
                        hy->m[k] = hy->dinv_h[k] * hy->w[k];
                        a3 = a3 + hy->w[k] * hy->u[k];
                    }
                    pt4[4 * t + 3] = a3;
                });
                for (int k = 0; k < 4; ++k) {
                    g[k] = 0.0;
                    for (int t = 0; t < T; ++t)
                        g[k] = g[k] + pt4[4 * t + k];
                }
                // the next n moves once its SpMV is done (the host has read
                // pin_n, so it may be overwritten)
                PPCG_HIP(hipEventRecord(hy->ev_upd, st));
                PPCG_HIP(hipStreamWaitEvent(cs, hy->ev_upd, 0));
                PPCG_HIP(hipMemcpyAsync(pin_n, nnext, sizeof(double) * n, hipMemcpyDeviceToHost, cs));
                PPCG_HIP(hipEventRecord(hy->ev_copy, cs));
            }
            gamma_prev = gamma;
            alpha_prev = alpha;
            gamma = g[0];
            uu = g[1];
            rr = g[2];
            delta = g[3];
            ++it;
        }
        // nothing of this sequence may still read or write the buffers
        PPCG_HIP(hipStreamSynchronize(cs));
        PPCG_HIP(hipStreamSynchronize(st));
        if (status == PPCG_BREAKDOWN && o.fixed_iters <= 0 && i > 0 && restarts < o.max_restarts &&
            it < o.max_iter) {
            ++restarts;
            continue;
        }
        if (status == PPCG_OK && o.fixed_iters <= 0 && o.stop == PPCG_STOP_REL_RESID) {
            double t2 = 0.0;
            PPCG_TRY(hybrid_resid_norm(hy, nullptr, &t2));
            const double rel = bnorm > 0 ? std::sqrt(t2) / bnorm : std::sqrt(t2);
            if (rel > o.tol) {
                if (restarts < o.max_restarts && it < o.max_iter) {
                    ++restarts;
                    continue;
                }
                status = PPCG_STAGNATED;
            }
        }
        break;
    }
    PPCG_HIP(hipMemcpy(x, hy->dx, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (info) {
        memset((char *)info + sizeof(size_t), 0, sizeof(ppcg_info) - sizeof(size_t));
        info->status = (ppcg_status)status;
        info->iters = it;
        info->restarts = restarts;
        info->rel_resid_recur = bnorm > 0 ? std::sqrt(rr) / bnorm : std::sqrt(rr);
        info->precond_norm = std::sqrt(uu);
        info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
        double t2 = 0.0;
        PPCG_TRY(hybrid_resid_norm(hy, nullptr, &t2));
        info->rel_resid_true = bnorm > 0 ? std::sqrt(t2) / bnorm : std::sqrt(t2);
        info->precision = PPCG_FP64;
        info->method = PPCG_METHOD_PIPECG;
    }
    return (ppcg_status)status;
}

}  // namespace

extern "C" {

ppcg_status ppcg_hybrid_destroy(ppcg_hybrid *hy)
{
    clear_error();
    if (!hy)
        return PPCG_OK;
    if (hy->stream)
        (void)hipStreamSynchronize(hy->stream);
    if (hy->gs)
        ppcg_shard_destroy(hy->gs);
    hy->arena.release();
    if (hy->pin_to_host) (void)host_free(hy->pin_to_host);
    if (hy->pin_to_dev) (void)host_free(hy->pin_to_dev);
    if (hy->pin_red) (void)host_free(hy->pin_red);
    if (hy->ev_halo) (void)hipEventDestroy(hy->ev_halo);
    if (hy->cstream) {
        (void)hipStreamSynchronize(hy->cstream);
        (void)hipStreamDestroy(hy->cstream);
    }
    if (hy->ev_upd) (void)hipEventDestroy(hy->ev_upd);
    if (hy->ev_copy) (void)hipEventDestroy(hy->ev_copy);
    if (hy->pin_vec) (void)host_free(hy->pin_vec);
    delete hy;
    return PPCG_OK;
}

ppcg_status ppcg_hybrid_create(const ppcg_csr *A, const ppcg_options *opt, ppcg_hybrid_scheme scheme,
                               int32_t host_threads, double cpu_share, void *hip_stream, ppcg_hybrid **out)
{
    clear_error();
    const bool task = scheme == PPCG_HYBRID_1 || scheme == PPCG_HYBRID_2;
    if (!out || !A || !opt || A->struct_size != sizeof(ppcg_csr) || opt->struct_size != sizeof(ppcg_options) ||
        A->mem != PPCG_MEM_HOST || A->n < 1 || A->nnz < A->n || A->nnz >= INT32_MAX || !A->row_ptr ||
        !A->col_idx || !A->values || host_threads < 1 || host_threads > 256 || !(cpu_share <= 1.0) ||
        !std::isfinite(cpu_share) || opt->precision != PPCG_FP64 || opt->method != PPCG_METHOD_PIPECG ||
        opt->vec_mem != PPCG_MEM_HOST || !(task || scheme == PPCG_HYBRID_3) || (task && cpu_share >= 0.0)) {
        set_error("invalid arguments (host CSR, FP64 PIPECG, host vectors, a scheme of ppcg_hybrid_scheme, "
                  "1..256 threads, cpu_share <= 1 for Hybrid-3 and < 0 for Hybrid-1/2)");
        return PPCG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    const int n = A->n;
    const int *rp = A->row_ptr, *ci = A->col_idx;
    const double *va = A->values;
    // validation and the Jacobi preconditioner (host copy of the diagonal)
    std::vector<double> dinv(n);
    if (rp[0] != 0 || rp[n] != A->nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[n] = nnz");
        return PPCG_ERR_BAD_CSR;
    }
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        bool found = false;
        if (rp[i + 1] < rp[i]) {
            set_error("row_ptr decreases at row %d", i);
            return PPCG_ERR_BAD_CSR;
        }
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n || !std::isfinite(va[k]) || (k > rp[i] && ci[k] <= ci[k - 1])) {
                set_error("row %d: bad column index or value", i);
                return PPCG_ERR_BAD_CSR;
            }
            if (ci[k] == i) {
                d = va[k];
                found = true;
            }
        }
        if (!found || !(d > 0.0)) {
            set_error("row %d: missing or non-positive diagonal", i);
            return PPCG_ERR_BAD_CSR;
        }
        dinv[i] = 1.0 / d;
    }
    std::unique_ptr<ppcg_hybrid> hy(new ppcg_hybrid());
    PPCG_HIP(hipGetDevice(&hy->device));
    hy->stream = (hipStream_t)hip_stream;
    hy->opt = *opt;
    hy->n = n;
    hy->scheme = scheme;
    hy->pool.reset(new HostPool(host_threads));
    // Performance model (Hybrid-3): five SpMVs over all of A on each side.
    if (!task) {
        ppcg_shard *full = nullptr;
        PPCG_TRY(ppcg_shard_create(A, 0, n, hip_stream, &full));
        std::unique_ptr<ppcg_shard, ppcg_status (*)(ppcg_shard *)> guard(full, ppcg_shard_destroy);
        double *dxv = nullptr, *dyv = nullptr;
        PPCG_HIP(hipMalloc(&dxv, sizeof(double) * n));
        PPCG_HIP(hipMalloc(&dyv, sizeof(double) * n));
        std::vector<double> ones(n, 1.0), yh(n);
        hipError_t e = hipMemcpy(dxv, ones.data(), sizeof(double) * n, hipMemcpyHostToDevice);
        double ms1 = 0.0, msg = 0.0, ms2 = 0.0;
        ppcg_status rc = e == hipSuccess ? ppcg_shard_time(full, dxv, dxv, dxv, dyv, 5, &ms1, &msg, &ms2)
                                         : PPCG_ERR_DEVICE;
        (void)dev_free(dxv);
        (void)dev_free(dyv);
        PPCG_TRY(rc);
        hy->t_gpu = ms1 * 1e-3;
        const int T = hy->pool->size();
        std::vector<int> lo(T + 1);
        for (int t = 0; t <= T; ++t)
            lo[t] = (int)((int64_t)n * t / T);
        const auto t0 = std::chrono::steady_clock::now();
        for (int rep = 0; rep < 5; ++rep)
            hy->pool->run([&](int t) {
                for (int i = lo[t]; i < lo[t + 1]; ++i) {
                    double a = 0.0;
                    for (int k = rp[i]; k < rp[i + 1]; ++k)
                        a = a + va[k] * ones[ci[k]];
                    yh[i] = a;
                }
            });
        hy->t_cpu = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / 5.0;
    }
    // Row split: the model's, or a forced share of the non-zeros; the
    // task-parallel schemes keep every row on the GPU.
    int32_t bounds[3];
    if (task) {
        bounds[1] = 0;
    } else if (cpu_share < 0.0) {
        const double times[2] = {hy->t_cpu, hy->t_gpu};
        PPCG_TRY(ppcg_split_rows(n, rp, 2, times, bounds));
    } else if (cpu_share == 0.0) {
        bounds[1] = 0;
    } else if (cpu_share == 1.0) {
        bounds[1] = n;
    } else {
        const double times[2] = {1.0 / cpu_share, 1.0 / (1.0 - cpu_share)};
        PPCG_TRY(ppcg_split_rows(n, rp, 2, times, bounds));
    }
    const int ncpu = bounds[1];
    hy->ncpu = ncpu;
    hy->ngpu = n - ncpu;
    // host thread ranges over the host rows
    const int T = hy->pool->size();
    hy->row_lo.resize(T + 1);
    for (int t = 0; t <= T; ++t)
        hy->row_lo[t] = (int)((int64_t)ncpu * t / T);
    // host part: 2-D decomposition of rows [0, ncpu)
    {
        std::vector<int> rem;
        for (int i = 0; i < ncpu; ++i)
            for (int k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] >= ncpu)
                    rem.push_back(ci[k]);
        std::sort(rem.begin(), rem.end());
        rem.erase(std::unique(rem.begin(), rem.end()), rem.end());
        hy->hcols = rem;
        hy->h1.rp.assign(ncpu + 1, 0);
        hy->h2.rp.assign(ncpu + 1, 0);
        for (int i = 0; i < ncpu; ++i) {
            for (int k = rp[i]; k < rp[i + 1]; ++k) {
                if (ci[k] < ncpu) {
                    hy->h1.ci.push_back(ci[k]);
                    hy->h1.val.push_back(va[k]);
                } else {
                    hy->h2.ci.push_back((int)(std::lower_bound(rem.begin(), rem.end(), ci[k]) - rem.begin()));
                    hy->h2.val.push_back(va[k]);
                }
            }
            hy->h1.rp[i + 1] = (int)hy->h1.ci.size();
            hy->h2.rp[i + 1] = (int)hy->h2.ci.size();
        }
        hy->dinv_h.assign(dinv.begin(), dinv.begin() + ncpu);
        for (auto *v : {&hy->x, &hy->r, &hy->u, &hy->w, &hy->m, &hy->nv, &hy->z, &hy->q, &hy->s, &hy->p, &hy->bh})
            v->assign(ncpu, 0.0);
    }
    // GPU part: shard of rows [ncpu, n) (its halo = the host-owned columns)
    const int ng = hy->ngpu;
    const int hc = (int)hy->hcols.size();
    if (ng > 0) {
        PPCG_TRY(ppcg_shard_create(A, ncpu, n, hip_stream, &hy->gs));
        hy->nblocks = (ng + kH3Threads - 1) / kH3Threads;
        const size_t vb = ((sizeof(double) * ng + 255) & ~(size_t)255);
        const size_t bytes = 13 * vb + ((sizeof(double) * 4 * hy->nblocks + 255) & ~(size_t)255) + 256 +
                             2 * (((sizeof(double) * (std::max(hy->gs->halo, hc) + 1)) + 255) & ~(size_t)255) +
                             ((sizeof(int) * (hc + 1) + 255) & ~(size_t)255);
        PPCG_TRY(hy->arena.alloc(bytes));
        double **vecs[] = {&hy->dx, &hy->dr, &hy->du, &hy->dw, &hy->dm, &hy->dn, &hy->dz,
                           &hy->dq, &hy->ds, &hy->dp, &hy->ddinv, &hy->db, &hy->dy};
        for (double **v : vecs)
            *v = (double *)hy->arena.take(sizeof(double) * ng);
        hy->dpart = (double *)hy->arena.take(sizeof(double) * 4 * hy->nblocks);
        hy->dred = (double *)hy->arena.take(sizeof(double) * 4);
        hy->dhalo = (double *)hy->arena.take(sizeof(double) * (hy->gs->halo + 1));
        hy->dpack = (double *)hy->arena.take(sizeof(double) * (hc + 1));
        hy->dhcols = (int *)hy->arena.take(sizeof(int) * (hc + 1));
        PPCG_HIP(hipMemcpy(hy->ddinv, dinv.data() + ncpu, sizeof(double) * ng, hipMemcpyHostToDevice));
        if (hc > 0)
            PPCG_HIP(hipMemcpy(hy->dhcols, hy->hcols.data(), sizeof(int) * hc, hipMemcpyHostToDevice));
    }
    PPCG_HIP(hipHostMalloc((void **)&hy->pin_to_host, sizeof(double) * (hc + 1), hipHostMallocDefault));
    PPCG_HIP(hipHostMalloc((void **)&hy->pin_to_dev, sizeof(double) * ((hy->gs ? hy->gs->halo : 0) + 1),
                           hipHostMallocDefault));
    PPCG_HIP(hipHostMalloc((void **)&hy->pin_red, sizeof(double) * 4, hipHostMallocDefault));
    PPCG_HIP(hipEventCreateWithFlags(&hy->ev_halo, hipEventDisableTiming));
    if (task) {
        // host thread ranges over all rows, the copy stream (default
        // priority) and the pinned vectors: w, r, u (Hybrid-1) or n (Hybrid-2)
        hy->full_lo.resize(T + 1);
        for (int t = 0; t <= T; ++t)
            hy->full_lo[t] = (int)((int64_t)n * t / T);
        PPCG_HIP(hipStreamCreateWithFlags(&hy->cstream, hipStreamNonBlocking));
        PPCG_HIP(hipEventCreateWithFlags(&hy->ev_upd, hipEventDisableTiming));
        PPCG_HIP(hipEventCreateWithFlags(&hy->ev_copy, hipEventDisableTiming));
        const int nvec = scheme == PPCG_HYBRID_1 ? 3 : 1;
        PPCG_HIP(hipHostMalloc((void **)&hy->pin_vec, sizeof(double) * (size_t)nvec * n, hipHostMallocDefault));
        if (scheme == PPCG_HYBRID_2) {
            hy->dinv_h = dinv;
            for (auto *v : {&hy->r, &hy->u, &hy->w, &hy->m, &hy->z, &hy->q, &hy->s})
                v->assign(n, 0.0);
        }
    }
    *out = hy.release();
    return PPCG_OK;
}

ppcg_status ppcg_hybrid_get_info(const ppcg_hybrid *hy, ppcg_hybrid_info *info)
{
    clear_error();
    if (!hy || !info || info->struct_size != sizeof(ppcg_hybrid_info)) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    info->n_cpu = hy->ncpu;
    info->n_gpu = hy->ngpu;
    info->host_threads = hy->pool->size();
    info->t_cpu_spmv_ms = hy->t_cpu * 1e3;
    info->t_gpu_spmv_ms = hy->t_gpu * 1e3;
    info->nnz_cpu_local = (int64_t)hy->h1.ci.size();
    info->nnz_cpu_remote = (int64_t)hy->h2.ci.size();
    info->nnz_gpu_local = hy->gs ? hy->gs->nnz1 : 0;
    info->nnz_gpu_remote = hy->gs ? hy->gs->nnz2 : 0;
    info->halo_to_cpu = (int32_t)hy->hcols.size();
    info->halo_to_gpu = hy->gs ? hy->gs->halo : 0;
    info->scheme = (ppcg_hybrid_scheme)hy->scheme;
    info->copy_bytes_per_iter = hy->scheme == PPCG_HYBRID_1   ? 3.0 * 8.0 * hy->n
                                : hy->scheme == PPCG_HYBRID_2 ? 8.0 * hy->n
                                                              : 8.0 * (info->halo_to_cpu + info->halo_to_gpu);
    return PPCG_OK;
}

ppcg_status ppcg_hybrid_solve(ppcg_hybrid *hy, const double *b, const double *x0, double *x, ppcg_info *info)
{
    clear_error();
    if (!hy || !b || !x || (info && info->struct_size != sizeof(ppcg_info))) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_HIP(hipSetDevice(hy->device));
    if (hy->scheme != PPCG_HYBRID_3)
        return solve_task(hy, b, x0, x, info);
    const auto t_begin = std::chrono::steady_clock::now();
    const int nc = hy->ncpu, ng = hy->ngpu, hc = (int)hy->hcols.size();
    const int T = hy->pool->size();
    hipStream_t st = hy->stream;
    const ppcg_options &o = hy->opt;
    const int g1 = (ng + kH3Threads - 1) / kH3Threads;
    std::vector<double> pt(T), pt4(4 * T);
    // inputs
    for (int i = 0; i < nc; ++i) {
        hy->bh[i] = b[i];
        hy->x[i] = x0 ? x0[i] : 0.0;
    }
    if (ng > 0) {
        PPCG_HIP(hipMemcpyAsync(hy->db, b + nc, sizeof(double) * ng, hipMemcpyHostToDevice, st));
        if (x0)
            PPCG_HIP(hipMemcpyAsync(hy->dx, x0 + nc, sizeof(double) * ng, hipMemcpyHostToDevice, st));
        else
            PPCG_HIP(hipMemsetAsync(hy->dx, 0, sizeof(double) * ng, st));
    }
    double bb = host_dot_rows(hy, hy->bh, hy->bh, pt);
    {
        // (b, b) on the GPU rows, reduced on the device
        std::vector<double> bg(ng);
        if (ng > 0) {
            PPCG_HIP(hipMemcpyAsync(bg.data(), hy->db, sizeof(double) * ng, hipMemcpyDeviceToHost, st));
            PPCG_HIP(hipStreamSynchronize(st));
        }
        double a = 0.0;
        for (int i = 0; i < ng; ++i)
            a = a + bg[i] * bg[i];
        bb = bb + a;
    }
    const double bnorm = std::sqrt(bb);
    int it = 0, restarts = 0, status = PPCG_OK;
    double gamma = 0, delta = 0, uu = 0, rr = 0, alpha_prev = 0, gamma_prev = 0, beta = 0;
    auto converged = [&]() {
        if (o.stop == PPCG_STOP_PRECOND_ABS)
            return std::sqrt(uu) < o.tol;
        return std::sqrt(rr) <= o.tol * bnorm;
    };
    // scalars: host partials (threads in order) + GPU partials
    auto combine = [&](const double *hp, int nvals) {
        double g[4] = {0, 0, 0, 0};
        for (int t = 0; t < T; ++t)
            for (int k = 0; k < nvals; ++k)
                g[k] = g[k] + hp[4 * t + k];
        for (int k = 0; k < nvals; ++k)
            g[k] = g[k] + (ng > 0 ? hy->pin_red[k] : 0.0);
        return std::vector<double>(g, g + 4);
    };
    for (;;) {
        // Algorithm 2 initialisation: r0 = b - A x0, u0 = M^-1 r0, w0 = A u0,
        // gamma0, delta0, (u,u), (r,r), m0 = M^-1 w0 (n0 is formed in the loop)
        {
            std::vector<double> yh(nc);
            PPCG_TRY(hybrid_spmv(hy, hy->x.data(), hy->dx, yh.data(), hy->dy));
            if (ng > 0)
                k_h3_init1<<<(ng + 255) / 256, 256, 0, st>>>(ng, hy->db, hy->dy, hy->ddinv, hy->dr, hy->du, hy->dz,
                                                            hy->dq, hy->ds, hy->dp);
            hy->pool->run([&](int t) {
                for (int i = hy->row_lo[t]; i < hy->row_lo[t + 1]; ++i) {
                    hy->r[i] = hy->bh[i] - yh[i];
                    hy->u[i] = hy->dinv_h[i] * hy->r[i];
                    hy->z[i] = hy->q[i] = hy->s[i] = hy->p[i] = 0.0;
                }
            });
            PPCG_TRY(hybrid_spmv(hy, hy->u.data(), hy->du, hy->w.data(), hy->dw));
            if (ng > 0) {
                k_h3_init2<<<g1, kH3Threads, 0, st>>>(ng, hy->dr, hy->du, hy->dw, hy->ddinv, hy->dm, hy->dpart);
                k_h3_reduce<<<1, kH3RedThreads, 0, st>>>(g1, hy->dpart, hy->dred);
                PPCG_HIP(hipMemcpyAsync(hy->pin_red, hy->dred, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
            }
            hy->pool->run([&](int t) {
                double a[4] = {0, 0, 0, 0};
                for (int i = hy->row_lo[t]; i < hy->row_lo[t + 1]; ++i) {
                    hy->m[i] = hy->dinv_h[i] * hy->w[i];
                    a[0] = a[0] + hy->r[i] * hy->u[i];
                    a[1] = a[1] + hy->u[i] * hy->u[i];
                    a[2] = a[2] + hy->r[i] * hy->r[i];
                    a[3] = a[3] + hy->w[i] * hy->u[i];
                }
                for (int k = 0; k < 4; ++k)
                    pt4[4 * t + k] = a[k];
            });
            PPCG_HIP(hipStreamSynchronize(st));
            const std::vector<double> g = combine(pt4.data(), 4);
            gamma = g[0];
            uu = g[1];
            rr = g[2];
            delta = g[3];
        }
        int i;
        for (i = 0;; ++i) {
            if (o.fixed_iters > 0) {
                if (it >= o.fixed_iters || gamma == 0.0) {
                    status = PPCG_OK;
                    break;
                }
            } else {
                if (converged()) {
                    status = PPCG_OK;
                    break;
                }
                if (it >= o.max_iter) {
                    status = PPCG_NOT_CONVERGED;
                    break;
                }
            }
            double denom;
            if (i > 0) {
                beta = gamma / gamma_prev;
                denom = delta - beta * gamma / alpha_prev;
            } else {
                beta = 0.0;
                denom = delta;
            }
            const double alpha = gamma / denom;
            if (!(gamma > 0.0) || !(denom > 0.0) || !std::isfinite(alpha) || !std::isfinite(beta)) {
                status = PPCG_BREAKDOWN;
                break;
            }
            // 1. the m entries each side needs start moving
            if (ng > 0) {
                if (hc > 0) {
                    k_h3_pack<<<(hc + 255) / 256, 256, 0, st>>>(hc, hy->dhcols, nc, hy->dm, hy->dpack);
                    PPCG_HIP(hipMemcpyAsync(hy->pin_to_host, hy->dpack, sizeof(double) * hc, hipMemcpyDeviceToHost,
                                            st));
                }
                PPCG_HIP(hipEventRecord(hy->ev_halo, st));
                if (hy->gs->halo > 0) {
                    host_pack(hy, hy->m.data());
                    PPCG_HIP(hipMemcpyAsync(hy->dhalo, hy->pin_to_dev, sizeof(double) * hy->gs->halo,
                                            hipMemcpyHostToDevice, st));
                }
                // 2-5 on the GPU (stream order keeps q's use of the old m
                // before the copy of m is replaced: m changes only in step 5)
                k_h3_update1<<<g1, kH3Threads, 0, st>>>(ng, alpha, beta, hy->dm, hy->dq, hy->dw, hy->ds, hy->du,
                                                        hy->dp, hy->dx, hy->dr, hy->dpart);
                PPCG_TRY(shard_launch(hy->gs, 1, hy->dm, hy->dhalo, hy->dn, nullptr, nullptr));
                PPCG_TRY(shard_launch(hy->gs, 2, hy->dm, hy->dhalo, hy->dn, nullptr, nullptr));
                k_h3_update2<<<g1, kH3Threads, 0, st>>>(ng, alpha, beta, hy->dn, hy->dz, hy->dw, hy->dm, hy->ddinv,
                                                        hy->du, hy->dpart);
                k_h3_reduce<<<1, kH3RedThreads, 0, st>>>(g1, hy->dpart, hy->dred);
                PPCG_HIP(hipMemcpyAsync(hy->pin_red, hy->dred, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
                PPCG_HIP(hipGetLastError());
            }
            // 2-3 on the host rows
            hy->pool->run([&](int t) {
                double a0 = 0, a1 = 0, a2 = 0;
                for (int k = hy->row_lo[t]; k < hy->row_lo[t + 1]; ++k) {
                    hy->q[k] = hy->m[k] + beta * hy->q[k];
                    hy->s[k] = hy->w[k] + beta * hy->s[k];
                    hy->p[k] = hy->u[k] + beta * hy->p[k];
                    hy->x[k] = hy->x[k] + alpha * hy->p[k];
                    hy->r[k] = hy->r[k] - alpha * hy->s[k];
                    hy->u[k] = hy->u[k] - alpha * hy->q[k];
                    a0 = a0 + hy->r[k] * hy->u[k];
                    a1 = a1 + hy->u[k] * hy->u[k];
                    a2 = a2 + hy->r[k] * hy->r[k];
                }
                pt4[4 * t + 0] = a0;
                pt4[4 * t + 1] = a1;
                pt4[4 * t + 2] = a2;
                host_spmv_rows(hy, hy->row_lo[t], hy->row_lo[t + 1], hy->m.data(), nullptr, hy->nv.data(), true,
                               false);
            });
            // 4. part 2 once the GPU's m entries are in host memory; 5.
            if (ng > 0 && hc > 0)
                PPCG_HIP(hipEventSynchronize(hy->ev_halo));
            hy->pool->run([&](int t) {
                host_spmv_rows(hy, hy->row_lo[t], hy->row_lo[t + 1], hy->m.data(), hy->pin_to_host, hy->nv.data(),
                               false, true);
                double a3 = 0.0;
                for (int k = hy->row_lo[t]; k < hy->row_lo[t + 1]; ++k) {
                    hy->z[k] = hy->nv[k] + beta * hy->z[k];
                    hy->w[k] = hy->w[k] - alpha * hy->z[k];
                    hy->m[k] = hy->dinv_h[k] * hy->w[k];
                    a3 = a3 + hy->w[k] * hy->u[k];
                }
                pt4[4 * t + 3] = a3;
            });
            // 6. both sides' partial sums
            if (ng > 0)
                PPCG_HIP(hipStreamSynchronize(st));
            gamma_prev = gamma;
            alpha_prev = alpha;
            const std::vector<double> g = combine(pt4.data(), 4);
            gamma = g[0];
            uu = g[1];
            rr = g[2];
            delta = g[3];
            ++it;
        }
        if (status == PPCG_BREAKDOWN && o.fixed_iters <= 0 && i > 0 && restarts < o.max_restarts &&
            it < o.max_iter) {
            ++restarts;
            continue;
        }
        if (status == PPCG_OK && o.fixed_iters <= 0 && o.stop == PPCG_STOP_REL_RESID) {
            // true residual b - A x
            std::vector<double> yh(nc);
            PPCG_TRY(hybrid_spmv(hy, hy->x.data(), hy->dx, yh.data(), hy->dy));
            double t2 = 0.0;
            for (int k = 0; k < nc; ++k) {
                const double d = hy->bh[k] - yh[k];
                t2 = t2 + d * d;
            }
            std::vector<double> yg(ng), bg(ng);
            if (ng > 0) {
                PPCG_HIP(hipMemcpy(yg.data(), hy->dy, sizeof(double) * ng, hipMemcpyDeviceToHost));
                PPCG_HIP(hipMemcpy(bg.data(), hy->db, sizeof(double) * ng, hipMemcpyDeviceToHost));
            }
            for (int k = 0; k < ng; ++k) {
                const double d = bg[k] - yg[k];
                t2 = t2 + d * d;
            }
            const double rel = bnorm > 0 ? std::sqrt(t2) / bnorm : std::sqrt(t2);
            if (rel > o.tol) {
                if (restarts < o.max_restarts && it < o.max_iter) {
                    ++restarts;
                    continue;
                }
                status = PPCG_STAGNATED;
            }
        }
        break;
    }
    // x out
    for (int k = 0; k < nc; ++k)
        x[k] = hy->x[k];
    if (ng > 0)
        PPCG_HIP(hipMemcpy(x + nc, hy->dx, sizeof(double) * ng, hipMemcpyDeviceToHost));
    if (info) {
        memset((char *)info + sizeof(size_t), 0, sizeof(ppcg_info) - sizeof(size_t));
        info->status = (ppcg_status)status;
        info->iters = it;
        info->restarts = restarts;
        info->rel_resid_recur = bnorm > 0 ? std::sqrt(rr) / bnorm : std::sqrt(rr);
        info->precond_norm = std::sqrt(uu);
        info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
        // the true residual of the returned x
        std::vector<double> yh(nc), xr(x, x + nc);
        PPCG_TRY(hybrid_spmv(hy, xr.data(), hy->dx, yh.data(), hy->dy));
        double t2 = 0.0;
        for (int k = 0; k < nc; ++k) {
            const double d = hy->bh[k] - yh[k];
            t2 = t2 + d * d;
        }
        std::vector<double> yg(ng), bg(ng);
        if (ng > 0) {
            PPCG_HIP(hipMemcpy(yg.data(), hy->dy, sizeof(double) * ng, hipMemcpyDeviceToHost));
            PPCG_HIP(hipMemcpy(bg.data(), hy->db, sizeof(double) * ng, hipMemcpyDeviceToHost));
        }
        for (int k = 0; k < ng; ++k) {
            const double d = bg[k] - yg[k];
            t2 = t2 + d * d;
        }
        info->rel_resid_true = bnorm > 0 ? std::sqrt(t2) / bnorm : std::sqrt(t2);
    }
    return (ppcg_status)status;
}

}  // extern "C"
