// ppcg_kernels.hpp -- HIP kernels of one PIPECG iteration for gfx950.
//
// The iteration of Algorithm 2 (Tiwari & Vadhiyar, Section III-B) runs as two
// launches over a table of (system, tile) work items:
//
//   k_vma   the eight vector recurrences z, q, s, p, x, r, u, w, the Jacobi
//           preconditioner m = M^-1 w and the partial sums of (r,u), (w,u),
//           (u,u), (r,r), all in one pass over the vectors (Section V-B:
//           fused VMAs with the preconditioner folded in).  Each workgroup
//           writes one partial per dot product.
//   k_spmv  n = A m (the SpMV), plus, in the designated workgroup of each
//           system (its tile 0), the fixed-order reduction of that system's
//           partials and the scalar recurrences: beta, alpha, the stopping
//           test and breakdown checks.  The reduction thus rides inside the
//           SpMV launch and the dot products cost no pass of their own.
//
// The same SpMV kernel, with other epilogues, performs the initialisation
// (r0 = b - A x0, u0 = M^-1 r0, w0 = A u0, m0 = M^-1 w0, n0 = A m0 and the
// initial dot products) and the true-residual pass b - A x.
//
// Arithmetic.  Every product and sum is rounded separately (this file is
// built with -ffp-contract=off), the SpMV sums each row in stored column
// order, and every reduction has a fixed order, so results are deterministic
// and, for a single system, identical run to run and alone or batched.
#pragma once

#include "ppcg_internal.hpp"

namespace ppcg {

enum SpmvMode : int {
    MODE_ITER = 0,   // nv = A m; reduce the fused-update partials; scalar update
    MODE_INIT1 = 1,  // r = b - A x; u = M^-1 r; partial (b,b); reset the state
    MODE_INIT2 = 2,  // w = A u; m = M^-1 w; partials (r,u),(w,u),(u,u),(r,r); reduce (b,b)
    MODE_RESID = 3,  // r = b - A x; partials (r,r), (b,b)
    MODE_PLAIN = 4   // nv = A x (timing only)
};

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Map the hardware workgroup id to a table position so that each of the 8
// XCDs (which receive workgroups round-robin) works on a contiguous range of
// tiles: neighbouring rows then share an L2, which serves the SpMV gathers.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    constexpr int X = 8;
    const int q = G / X, r = G % X;
    const int x = b % X, k = b / X;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = v + __shfl_xor(v, off, 64);
    return v;  // identical in every lane (each step adds a commuted pair)
}

// Sum NV values over the workgroup in a fixed order; result valid in thread 0.
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* [NT/64 * NV] */)
{
    constexpr int W = NT / 64;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            lds[wid * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = lds[k];
            for (int w = 1; w < W; ++w)
                a = a + lds[w * NV + k];
            v[k] = a;
        }
    }
}

// Reduce slot `slot` of a system's partials (ntiles x 4) in a fixed order.
// Every thread of the workgroup must call it; result valid in thread 0.
template <int NT>
__device__ __forceinline__ void reduce_partials(const SysDesc &d, int slot, double (&out)[kNumPartials],
                                                double *lds)
{
    const double *P = d.part + (size_t)slot * d.ntiles * kNumPartials;
#pragma unroll
    for (int k = 0; k < kNumPartials; ++k)
        out[k] = 0.0;
    for (int t = threadIdx.x; t < d.ntiles; t += NT) {
#pragma unroll
        for (int k = 0; k < kNumPartials; ++k)
            out[k] = out[k] + P[t * kNumPartials + k];
    }
    block_sum<NT, kNumPartials>(out, lds);
}

// Scalar recurrences and stopping test, executed by one thread per system
// after the dot products of an iteration (or of the initialisation) are
// reduced.  Mirrors the top of the loop of Algorithm 2: test convergence,
// then the iteration limit, then beta_i = gamma_i / gamma_{i-1} and
// alpha_i = gamma_i / (delta - beta_i gamma_i / alpha_{i-1}) (beta = 0 and
// alpha = gamma / delta on the first iteration of a start), with breakdown
// when gamma <= 0, the denominator <= 0 or a scalar is not finite.
__device__ inline void scalar_update(const SysDesc &d, SysState *st, const double (&v)[kNumPartials])
{
    if (st->phase) {
        st->phase = 0;
    } else {
        st->iter += 1;
        st->i_start += 1;
    }
    st->gen += 1;
    const double g = v[0], dl = v[1], uu = v[2], rr = v[3];
    st->gamma = g;
    st->delta = dl;
    st->uu = uu;
    st->rr = rr;
    bool conv;
    if (d.fixed > 0)
        conv = (st->iter >= d.fixed) || (g == 0.0);
    else if (d.stop == STOP_ABS)
        conv = sqrt(uu) < d.tol;
    else
        conv = sqrt(rr) <= d.tol * sqrt(st->bnorm2);
    if (conv) {
        st->done = 1;
        st->status = ST_OK;
        return;
    }
    if (d.fixed <= 0 && st->iter >= d.maxit) {
        st->done = 1;
        st->status = ST_NOT_CONVERGED;
        return;
    }
    double beta, denom;
    if (st->i_start > 0) {
        beta = g / st->gamma_prev;
        denom = dl - beta * g / st->alpha_prev;
    } else {
        beta = 0.0;
        denom = dl;
    }
    const double alpha = g / denom;
    if (!(g > 0.0) || !(denom > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
        st->done = 1;
        st->status = ST_BREAKDOWN;
        return;
    }
    st->alpha = alpha;
    st->beta = beta;
    st->gamma_prev = g;
    st->alpha_prev = alpha;
}

// ---------------------------------------------------------------------------
// Fused vector updates + Jacobi + dot-product partials.
template <typename T>
__device__ __forceinline__ void vma_elem(T sa, T sb, T nv, T &z, T m, T &q, T &w, T &s, T &u, T &p, T &x,
                                         T &r, T dinv, T &m_out, double (&acc)[kNumPartials])
{
    z = nv + sb * z;
    q = m + sb * q;
    s = w + sb * s;
    p = u + sb * p;
    x = x + sa * p;
    r = r - sa * s;
    u = u - sa * q;
    w = w - sa * z;
    m_out = dinv * w;
    const double rd = (double)r, ud = (double)u, wd = (double)w;
    acc[0] = acc[0] + rd * ud;
    acc[1] = acc[1] + wd * ud;
    acc[2] = acc[2] + ud * ud;
    acc[3] = acc[3] + rd * rd;
}

template <typename T>
__global__ __launch_bounds__(kVmaThreads) void k_vma(const WorkItem *__restrict__ table,
                                                     const int *__restrict__ count,
                                                     const SysDesc *__restrict__ descs, int remap)
{
    __shared__ double lds[kVmaThreads / 64 * kNumPartials];
    const int pos = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    const SysState *st = d.st;
    if (st->done)
        return;
    const T sa = (T)st->alpha, sb = (T)st->beta;
    const int n = d.n;
    T *__restrict__ X = (T *)d.x;
    T *__restrict__ R = (T *)d.r;
    T *__restrict__ U = (T *)d.u;
    T *__restrict__ W = (T *)d.w;
    T *__restrict__ M = (T *)d.m;
    const T *__restrict__ NV = (const T *)d.nv;
    T *__restrict__ Z = (T *)d.z;
    T *__restrict__ Q = (T *)d.q;
    T *__restrict__ S = (T *)d.s;
    T *__restrict__ P = (T *)d.p;
    const T *__restrict__ DI = (const T *)d.dinv;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    const int i = wi.tile * kTileRows + threadIdx.x * 2;
    using V2 = typename Vec2<T>::type;
    if (i + 1 < n) {
        V2 nv = *(const V2 *)(NV + i), z = *(const V2 *)(Z + i), m = *(const V2 *)(M + i);
        V2 q = *(const V2 *)(Q + i), w = *(const V2 *)(W + i), s = *(const V2 *)(S + i);
        V2 u = *(const V2 *)(U + i), p = *(const V2 *)(P + i), x = *(const V2 *)(X + i);
        V2 r = *(const V2 *)(R + i), di = *(const V2 *)(DI + i);
        V2 mo;
        vma_elem<T>(sa, sb, nv.x, z.x, m.x, q.x, w.x, s.x, u.x, p.x, x.x, r.x, di.x, mo.x, acc);
        vma_elem<T>(sa, sb, nv.y, z.y, m.y, q.y, w.y, s.y, u.y, p.y, x.y, r.y, di.y, mo.y, acc);
        *(V2 *)(Z + i) = z;
        *(V2 *)(Q + i) = q;
        *(V2 *)(S + i) = s;
        *(V2 *)(P + i) = p;
        *(V2 *)(X + i) = x;
        *(V2 *)(R + i) = r;
        *(V2 *)(U + i) = u;
        *(V2 *)(W + i) = w;
        *(V2 *)(M + i) = mo;
    } else if (i < n) {
        T z = Z[i], q = Q[i], w = W[i], s = S[i], u = U[i], p = P[i], x = X[i], r = R[i], mo;
        vma_elem<T>(sa, sb, NV[i], z, M[i], q, w, s, u, p, x, r, DI[i], mo, acc);
        Z[i] = z; Q[i] = q; S[i] = s; P[i] = p; X[i] = x; R[i] = r; U[i] = u; W[i] = w; M[i] = mo;
    }
    block_sum<kVmaThreads, kNumPartials>(acc, lds);
    if (threadIdx.x == 0) {
        double *out = d.part + ((size_t)d.ntiles + wi.tile) * kNumPartials;  // slot 1
#pragma unroll
        for (int k = 0; k < kNumPartials; ++k)
            out[k] = acc[k];
    }
}

// ---------------------------------------------------------------------------
// SpMV row kernels.

// SELL-C-sigma, C = 64, one lane per row, chunk-major storage: entry k of
// row (chunk c, lane l) is at cptr[c] + k * 64 + l.  Rows are summed in
// stored (ascending original column) order.
template <typename T>
__device__ __forceinline__ T sell_row(const int64_t *__restrict__ cptr, const int *__restrict__ col,
                                      const T *__restrict__ val, const T *__restrict__ xin, int chunk,
                                      int lane)
{
    const int64_t base = cptr[chunk];
    const int len = (int)((cptr[chunk + 1] - base) / kSellC);
    const int *c = col + base + lane;
    const T *v = val + base + lane;
    T acc = (T)0;
#pragma unroll 4
    for (int k = 0; k < len; ++k)
        acc = acc + v[(size_t)k * kSellC] * xin[c[(size_t)k * kSellC]];
    return acc;
}

// Per-row epilogue of each mode.  Returns nothing; accumulates partials.
template <typename T, int MODE>
__device__ __forceinline__ void spmv_epilogue(const SysDesc &d, int i, T y, double (&acc)[kNumPartials])
{
    if (MODE == MODE_ITER || MODE == MODE_PLAIN) {
        ((T *)d.nv)[i] = y;
    } else if (MODE == MODE_INIT1) {
        const T bi = ((const T *)d.b)[i];
        const T ri = bi - y;
        const T ui = ((const T *)d.dinv)[i] * ri;
        ((T *)d.r)[i] = ri;
        ((T *)d.u)[i] = ui;
        acc[0] = acc[0] + (double)bi * (double)bi;
    } else if (MODE == MODE_INIT2) {
        const T ri = ((const T *)d.r)[i];
        const T ui = ((const T *)d.u)[i];
        const T mi = ((const T *)d.dinv)[i] * y;
        ((T *)d.w)[i] = y;
        ((T *)d.m)[i] = mi;
        const double rd = (double)ri, ud = (double)ui, wd = (double)y;
        acc[0] = acc[0] + rd * ud;
        acc[1] = acc[1] + wd * ud;
        acc[2] = acc[2] + ud * ud;
        acc[3] = acc[3] + rd * rd;
    } else if (MODE == MODE_RESID) {
        const T bi = ((const T *)d.b)[i];
        const T ti = bi - y;
        ((T *)d.r)[i] = ti;
        acc[0] = acc[0] + (double)ti * (double)ti;
        acc[1] = acc[1] + (double)bi * (double)bi;
    }
}

template <int MODE> struct SpmvIO;
template <> struct SpmvIO<MODE_ITER> { static __device__ const void *in(const SysDesc &d) { return d.m; } };
template <> struct SpmvIO<MODE_PLAIN> { static __device__ const void *in(const SysDesc &d) { return d.x; } };
template <> struct SpmvIO<MODE_INIT1> { static __device__ const void *in(const SysDesc &d) { return d.x; } };
template <> struct SpmvIO<MODE_INIT2> { static __device__ const void *in(const SysDesc &d) { return d.u; } };
template <> struct SpmvIO<MODE_RESID> { static __device__ const void *in(const SysDesc &d) { return d.x; } };

template <typename T, int MODE>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv(const WorkItem *__restrict__ table,
                                                       const int *__restrict__ count,
                                                       const SysDesc *__restrict__ descs, int remap)
{
    __shared__ double lds[kSpmvThreads / 64 * kNumPartials];
    const int pos = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    SysState *st = d.st;
    if (MODE == MODE_ITER && st->done)
        return;
    const T *__restrict__ xin = (const T *)SpmvIO<MODE>::in(d);
    const T *__restrict__ val = (const T *)d.val;
    const int n = d.n;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    if (d.fmt == FMT_SELL) {
        const int lane = threadIdx.x & 63;
        const int chunk = wi.tile * kSellChunksPerTile + (threadIdx.x >> 6);
        const int i = chunk * kSellC + lane;
        if (chunk * kSellC < n) {
            const T y = sell_row<T>(d.cptr, d.col, val, xin, chunk, lane);
            if (i < n)
                spmv_epilogue<T, MODE>(d, i, y, acc);
        }
    } else {
        // CSR-vector: groups of L lanes per row, L a power of two in [2, 64];
        // lane k of a group sums entries k, k + L, ...; the group then
        // combines its lanes with a butterfly.
        const int L = d.lanes;
        const int g = threadIdx.x / L, l = threadIdx.x % L;
        const int rows_per_pass = kSpmvThreads / L;
        const int *__restrict__ rp = d.rp;
        const int *__restrict__ col = d.col;
        for (int pass = 0; pass < L; ++pass) {
            const int i = wi.tile * kTileRows + pass * rows_per_pass + g;
            T a = (T)0;
            if (i < n) {
                const int e = rp[i + 1];
                for (int k = rp[i] + l; k < e; k += L)
                    a = a + val[k] * xin[col[k]];
            }
            for (int off = L >> 1; off >= 1; off >>= 1)
                a = a + __shfl_xor(a, off, 64);
            if (l == 0 && i < n)
                spmv_epilogue<T, MODE>(d, i, a, acc);
        }
    }
    if (MODE == MODE_INIT1 || MODE == MODE_INIT2 || MODE == MODE_RESID) {
        double v[kNumPartials] = {acc[0], acc[1], acc[2], acc[3]};
        block_sum<kSpmvThreads, kNumPartials>(v, lds);
        if (threadIdx.x == 0) {
            const int slot = (MODE == MODE_INIT2) ? 1 : 0;
            double *out = d.part + ((size_t)slot * d.ntiles + wi.tile) * kNumPartials;
#pragma unroll
            for (int k = 0; k < kNumPartials; ++k)
                out[k] = v[k];
        }
    }
    if (wi.tile != 0)
        return;
    // Designated workgroup of this system.
    if (MODE == MODE_INIT1) {
        if (threadIdx.x == 0) {
            st->phase = 1;
            st->i_start = 0;
            st->done = 0;
            st->status = ST_OK;
        }
    } else if (MODE == MODE_INIT2 || MODE == MODE_ITER) {
        __syncthreads();  // lds reuse
        double v[kNumPartials];
        reduce_partials<kSpmvThreads>(d, MODE == MODE_INIT2 ? 0 : 1, v, lds);
        if (threadIdx.x == 0) {
            if (MODE == MODE_INIT2)
                st->bnorm2 = v[0];
            else
                scalar_update(d, st, v);
        }
    }
}

// Reduce the true-residual partials of each system (tile-0 workgroups only).
__global__ __launch_bounds__(kSpmvThreads) void k_reduce_resid(const WorkItem *__restrict__ table,
                                                               const int *__restrict__ count,
                                                               const SysDesc *__restrict__ descs)
{
    __shared__ double lds[kSpmvThreads / 64 * kNumPartials];
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    if (wi.tile != 0)
        return;
    const SysDesc &d = descs[wi.slot];
    double v[kNumPartials];
    reduce_partials<kSpmvThreads>(d, 0, v, lds);
    if (threadIdx.x == 0) {
        d.st->tnorm2 = v[0];
        d.st->bnorm2 = v[1];
    }
}

// Mixed precision, start of an inner solve: b32 = r64 / ||r64||, x32 = 0.
// Work items name FP64 slots; SysDesc::pair is the FP32 slot of the system.
__global__ void k_mix_start(const WorkItem *__restrict__ table, const int *__restrict__ count,
                            const SysDesc *__restrict__ d64, const SysDesc *__restrict__ d32)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &a = d64[wi.slot];
    const SysDesc &f = d32[a.pair];
    const double inv = 1.0 / sqrt(a.st->tnorm2);
    const double *__restrict__ r = (const double *)a.r;
    float *__restrict__ b32 = (float *)f.b;
    float *__restrict__ x32 = (float *)f.x;
    for (int k = threadIdx.x; k < kTileRows; k += blockDim.x) {
        const int i = wi.tile * kTileRows + k;
        if (i < a.n) {
            b32[i] = (float)(r[i] * inv);
            x32[i] = 0.0f;
        }
    }
}

// Mixed precision, end of an inner solve: x64 += ||r64|| * x32.
__global__ void k_mix_correct(const WorkItem *__restrict__ table, const int *__restrict__ count,
                              const SysDesc *__restrict__ d64, const SysDesc *__restrict__ d32)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &a = d64[wi.slot];
    const SysDesc &f = d32[a.pair];
    const double rn = sqrt(a.st->tnorm2);
    double *__restrict__ x = (double *)a.x;
    const float *__restrict__ x32 = (const float *)f.x;
    for (int k = threadIdx.x; k < kTileRows; k += blockDim.x) {
        const int i = wi.tile * kTileRows + k;
        if (i < a.n)
            x[i] = x[i] + rn * (double)x32[i];
    }
}

// ---------------------------------------------------------------------------
// Small elementwise kernels used around the solve.

// out[p] = in[perm[p]] (perm == nullptr: plain copy).
template <typename TO, typename TI>
__global__ void k_gather(int n, const int *__restrict__ perm, const TI *__restrict__ in, TO *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = (TO)in[perm ? perm[i] : i];
}

// out[perm[p]] = in[p] (perm == nullptr: plain copy).
__global__ void k_scatter(int n, const int *__restrict__ perm, const double *__restrict__ in,
                          double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[perm ? perm[i] : i] = in[i];
}

template <typename T>
__global__ void k_fill(size_t n, T *__restrict__ out, T v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = v;
}

}  // namespace ppcg
