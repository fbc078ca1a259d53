// ppcg_kernels.hpp -- HIP kernels of one PIPECG iteration for gfx950.
//
// The iteration of Algorithm 2 (Tiwari & Vadhiyar, Section III-B) runs as two
// launches over a table of (system, tile) work items:
//
//   k_vma   the vector recurrences of z, s, p, x, r, w, the Jacobi
//           preconditioner m = M^-1 w and the partial sums of (r,u), (w,u),
//           (u,u), (r,r), all in one pass over the vectors (Section V-B:
//           fused VMAs with the preconditioner folded in).  With a diagonal
//           M, u = M^-1 r and q = M^-1 s are formed from r and s instead of
//           being carried as vectors, and x-updates are applied two at a
//           time (see vma_elem).  Each workgroup writes one partial per dot
//           product.
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

#include <type_traits>

#include "ppcg_internal.hpp"

namespace ppcg {

enum SpmvMode : int {
    MODE_ITER = 0,   // nv = A m; reduce the fused-update partials; scalar update
    MODE_INIT1 = 1,  // r = b - A x; u = M^-1 r; partial (b,b); reset the state
    MODE_INIT2 = 2,  // w = A u; m = M^-1 w; partials (r,u),(w,u),(u,u),(r,r); reduce (b,b)
    MODE_RESID = 3,  // r = b - A x; partials (r,r), (b,b)
    MODE_PLAIN = 4,  // nv = A x (timing only)
    // Residual replacement (reliable update) against the FP64 operator:
    MODE_REPL1 = 5,  // r = b - A x (FP64 values); u = M^-1 r
    MODE_DUAL1 = 6,  // w = A u and s = A p in one pass; m = M^-1 w; q = M^-1 s;
                     // partials (r,u),(w,u),(u,u),(r,r),(u,s),(p,s)
    MODE_DUAL2 = 7,  // nv = A m and z = A q in one pass; reduce; scalars with the
                     // exact alpha denominator
    MODE_INIT0 = 8   // MODE_INIT1 for x = 0 (r = b exactly: A 0 sums to +0 in every
                     // row), without the pass over the matrix
};

constexpr int kReplPartials = 6;

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = dvec2; };
template <> struct Vec2<float> { using type = fvec2; };

// The vectors and matrix arrays reach the kernels as generic pointers (from
// the system descriptor), for which the compiler emits flat loads and
// stores.  Every such buffer is device or pinned host memory, never LDS or
// scratch, so the hot kernels cast them to the global address space and get
// global_load / global_store: no aperture check, and no share of the counter
// that scalar loads and LDS accesses wait on.
#ifndef PPCG_GLOBAL_AS
#define PPCG_GLOBAL_AS 1
#endif
#if PPCG_GLOBAL_AS
#define PPCG_AS1 __attribute__((address_space(1)))
#else
#define PPCG_AS1
#endif
template <typename T>
__device__ __forceinline__ PPCG_AS1 T *as_global(T *p)
{
    return (PPCG_AS1 T *)p;
}

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

// v of the lane that the DPP pattern CTRL names (within the lane's row of 16).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the wavefront: a butterfly over lane pairs at distance 32, 16,
// 8, 4, 2, 1; each step adds a commuted pair, so the result is identical in
// every lane.  The first two steps cross rows of 16 lanes (LDS permutes); the
// other four stay inside a row and use DPP moves (a short dependency chain).
// Rotating a row by 8 reaches lane i ^ 8; rotating it by 4 reaches i ^ 4 or
// i ^ 4 ^ 8, which hold the same value once the distance-8 step is done; the
// quad permutations reach i ^ 2 and i ^ 1 exactly.  So the sums are those of
// the plain distance-32..1 butterfly, bit for bit.
__device__ __forceinline__ double wave_sum(double v)
{
    v = v + __shfl_xor(v, 32, 64);
    v = v + __shfl_xor(v, 16, 64);
    v = v + dpp_f64<0x128>(v);  // row_ror:8
    v = v + dpp_f64<0x124>(v);  // row_ror:4
    v = v + dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]: lane i ^ 2
    v = v + dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]: lane i ^ 1
    return v;
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
template <int NT, int NV = kNumPartials>
__device__ __forceinline__ void reduce_partials(const SysDesc &d, int slot, double (&out)[NV], double *lds)
{
    const PPCG_AS1 double *P = as_global(d.part + (size_t)slot * d.ntiles * kPartStride);
#pragma unroll
    for (int k = 0; k < NV; ++k)
        out[k] = 0.0;
    // Batches of 2 tiles per thread: loads first, then the sums in tile order.
    for (int t0 = threadIdx.x; t0 < d.ntiles; t0 += 2 * NT) {
        double v[2][NV];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int t = t0 + j * NT;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                v[j][k] = t < d.ntiles ? P[(size_t)t * kPartStride + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (t0 + j * NT < d.ntiles) {
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    out[k] = out[k] + v[j][k];
            }
    }
    block_sum<NT, NV>(out, lds);
}

// Scalar recurrences and stopping test, executed by one thread per system
// after the dot products of an iteration (or of the initialisation) are
// reduced.  Mirrors the top of the loop of Algorithm 2: test convergence,
// then the iteration limit, then beta_i = gamma_i / gamma_{i-1} and
// alpha_i = gamma_i / (delta - beta_i gamma_i / alpha_{i-1}) (beta = 0 and
// alpha = gamma / delta on the first iteration of a start), with breakdown
// when gamma <= 0, the denominator <= 0 or a scalar is not finite.
//
// FP32-values mode (d.vals32) differs in two ways.  (1) The denominator
// (p_i, A p_i) is evaluated directly, (p, A p) = delta + 2 beta (u, s_{i-1})
// + beta^2 (p_{i-1}, s_{i-1}) with A symmetric, from two extra dot products
// of the fused update (v[4], v[5]): the recurrence form relies on CG
// orthogonality identities that a residual computed with the FP64 operator
// does not satisfy for the FP32-valued recurrences.  (2) Once the residual
// has fallen by d.repl_factor since the last start or reliable update, the
// system pauses (ST_REPLACE) so the host can run the reliable update.
template <int NV>
__device__ inline void scalar_update(const SysDesc &d, SysState *st, const double (&v)[NV])
{
    const bool first = st->phase != 0;
    if (st->phase) {
        st->phase = 0;
    } else {
        st->iter += 1;
        st->i_start += 1;
    }
    st->gamma_prev2 = st->gamma_prev;
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
    if constexpr (NV >= kReplPartials) {
        if (d.vals32) {
            const double rn = sqrt(rr);
            if (first) {
                st->repl_ref = rn;
            } else if (d.repl_factor > 0.0 && rn < d.repl_factor * st->repl_ref) {
                st->done = 1;
                st->status = ST_REPLACE;
                return;
            }
        }
    }
    double beta, denom;
    if (st->i_start > 0) {
        beta = g / st->gamma_prev;
        if constexpr (NV >= kReplPartials)
            denom = d.vals32 ? dl + 2.0 * beta * v[4] + beta * beta * v[5] : dl - beta * g / st->alpha_prev;
        else
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

// Scalars after a residual replacement.  r, u, w, m, n were recomputed from
// the FP64 residual and s, q, z from the current direction p, so the
// recurrence for alpha's denominator (p, A p) = delta - beta gamma /
// alpha_{i-1} no longer holds exactly; it is evaluated directly instead:
// with p' = u + beta p and A p' = w + beta s, and A symmetric,
//   (p', A p') = (u, w) + 2 beta (u, s) + beta^2 (p, s).
// The iteration counters do not move.
__device__ inline void scalar_update_repl(const SysDesc &d, SysState *st, const double (&v)[kReplPartials])
{
    const double g = v[0], dl = v[1], uu = v[2], rr = v[3], us = v[4], ps = v[5];
    st->gamma = g;
    st->delta = dl;
    st->uu = uu;
    st->rr = rr;
    st->done = 0;
    st->status = ST_OK;
    bool conv;
    if (d.fixed > 0)
        conv = (st->iter >= d.fixed) || (g == 0.0);
    else if (d.stop == STOP_ABS)
        conv = sqrt(uu) < d.tol;
    else
        conv = sqrt(rr) <= d.tol * sqrt(st->bnorm2);
    if (conv) {
        st->done = 1;
        return;
    }
    if (d.fixed <= 0 && st->iter >= d.maxit) {
        st->done = 1;
        st->status = ST_NOT_CONVERGED;
        return;
    }
    st->repl_ref = sqrt(rr);
    double beta = 0.0, denom = dl;
    if (st->i_start > 0) {
        beta = g / st->gamma_prev2;
        denom = dl + 2.0 * beta * us + beta * beta * ps;
        if (!(denom > 0.0)) {
            // The kept direction is no longer usable: restart the direction
            // (beta = 0) from the replaced residual instead of breaking down.
            st->i_start = 0;
            beta = 0.0;
            denom = dl;
        }
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
//
// With the Jacobi preconditioner M^-1 is a diagonal scaling, so three of
// Algorithm 2's preconditioned vectors are the scaled unpreconditioned ones
// at every step: m_i = M^-1 w_i, u_i = M^-1 r_i and q_i = M^-1 s_i.  (Each
// holds after the initialisation, where q_0 = m_0 and s_0 = w_0, and is kept
// by the updates: q_i = m_i + beta q_{i-1} = M^-1 (w_i + beta s_{i-1}), and
// u_{i+1} = u_i - alpha q_i = M^-1 (r_i - alpha s_i).)  The kernel therefore
// forms u from r with the inverse diagonal instead of carrying u and q as
// vectors of their own: neither is read and q is never stored, four vector
// streams fewer.  m, which the SpMV gathers, is still stored.  Every writer
// of r (the initialisation, a reliable update, this kernel) also writes
// u = dinv * r, so the u read back elsewhere is the same rounded product.
// In exact arithmetic the iterates are Algorithm 2's; in floating point the
// two recurrences for u and q are replaced by the exact scaling.
//
// x is not needed by the iteration itself, so its update x += alpha p is
// left to the caller: k_vma defers every other one and applies two at once
// (x + alpha_{i-1} p_{i-1}, then + alpha_i p_i: the same two rounded
// operations as one at a time), so x is read and written every other launch.
template <typename T, int NV>
__device__ __forceinline__ void vma_elem(T sa, T sb, T nv, T &z, T &w, T &s, T &p, T &r, T dinv, T &u_out,
                                         T &m_out, double (&acc)[NV])
{
    const T u = dinv * r;  // u_i
    z = nv + sb * z;
    s = w + sb * s;
    p = u + sb * p;
    r = r - sa * s;
    w = w - sa * z;
    u_out = dinv * r;  // u_{i+1}
    m_out = dinv * w;  // m_{i+1}
    const double rd = (double)r, ud = (double)u_out, wd = (double)w;
    acc[0] = acc[0] + rd * ud;
    acc[1] = acc[1] + wd * ud;
    acc[2] = acc[2] + ud * ud;
    acc[3] = acc[3] + rd * rd;
    if constexpr (NV >= kReplPartials) {
        const double sd = (double)s, pd = (double)p;
        acc[4] = acc[4] + ud * sd;
        acc[5] = acc[5] + pd * sd;
    }
}

#ifndef PPCG_VMA_NT
#define PPCG_VMA_NT 0
#endif

template <typename V>
__device__ __forceinline__ V vload(const PPCG_AS1 V *p)
{
#if PPCG_VMA_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <typename V>
__device__ __forceinline__ void vstore(PPCG_AS1 V *p, V v)
{
#if PPCG_VMA_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// EXACT: also emit the partials of (u_{i+1}, s_i) and (p_i, s_i) for the
// directly evaluated alpha denominator (FP32-values mode).
template <typename T, bool EXACT = false>
__global__ __launch_bounds__(kVmaThreads) void k_vma(const WorkItem *__restrict__ table,
                                                     const int *__restrict__ count,
                                                     const SysDesc *__restrict__ descs, int remap)
{
    constexpr int NV = EXACT ? kReplPartials : kNumPartials;
    __shared__ double lds[kVmaThreads / 64 * NV];
    // Graphs bake a grid that may exceed the live table: blocks past it exit,
    // and the XCD-aware order is taken over the live items only, so that
    // every XCD gets an equal share of them.
    const int live = *count;
    if ((int)blockIdx.x >= live)
        return;
    const int pos = remap ? xcd_remap(blockIdx.x, live) : (int)blockIdx.x;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    const SysState *st = d.st;
    if (st->done)
        return;
    const T sa = (T)st->alpha, sb = (T)st->beta;
    // x_pending: x still lacks alpha_{i-1} p_{i-1}; apply it with this
    // iteration's term.  Otherwise defer this iteration's term (x untouched).
    const bool xp = st->x_pending != 0;
    const T ax = (T)st->alpha_x;
    const int n = d.n;
    PPCG_AS1 T *__restrict__ X = as_global((T *)d.x);
    PPCG_AS1 T *__restrict__ R = as_global((T *)d.r);
    PPCG_AS1 T *__restrict__ W = as_global((T *)d.w);
    PPCG_AS1 T *__restrict__ M = as_global((T *)d.m);
    const PPCG_AS1 T *__restrict__ NVv = as_global((const T *)d.nv);
    PPCG_AS1 T *__restrict__ Z = as_global((T *)d.z);
    PPCG_AS1 T *__restrict__ S = as_global((T *)d.s);
    PPCG_AS1 T *__restrict__ P = as_global((T *)d.p);
    const PPCG_AS1 T *__restrict__ DI = as_global((const T *)d.dinv);
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k)
        acc[k] = 0.0;
    const int i = wi.tile * kTileRows + threadIdx.x * 2;
    using V2 = typename Vec2<T>::type;
    if (i + 1 < n) {
        using CV2 = const PPCG_AS1 V2;
        V2 nv = vload((CV2 *)(NVv + i)), z = vload((CV2 *)(Z + i)), w = vload((CV2 *)(W + i));
        V2 s = vload((CV2 *)(S + i)), p = vload((CV2 *)(P + i));
        // a constant diagonal: every lane reads dinv[0..1] (one cached line)
        V2 r = vload((CV2 *)(R + i)), di = vload((CV2 *)(DI + (d.dinv_const ? 0 : i)));
        V2 x;
        if (xp)
            x = vload((CV2 *)(X + i));
        V2 mo;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const T pold = p[j];
            T zj = z[j], wj = w[j], sj = s[j], pj = p[j], rj = r[j], uj, mj;
            vma_elem<T, NV>(sa, sb, nv[j], zj, wj, sj, pj, rj, di[j], uj, mj, acc);
            z[j] = zj; w[j] = wj; s[j] = sj; p[j] = pj; r[j] = rj; mo[j] = mj;
            if (xp) {
                const T x1 = x[j] + ax * pold;
                x[j] = x1 + sa * pj;
            }
        }
        using GV2 = PPCG_AS1 V2;
        vstore((GV2 *)(Z + i), z);
        vstore((GV2 *)(S + i), s);
        vstore((GV2 *)(P + i), p);
        if (xp)
            vstore((GV2 *)(X + i), x);
        vstore((GV2 *)(R + i), r);
        vstore((GV2 *)(W + i), w);
        vstore((GV2 *)(M + i), mo);
    } else if (i < n) {
        T z = Z[i], w = W[i], s = S[i], p = P[i], r = R[i], u, mo;
        const T pold = p;
        vma_elem<T, NV>(sa, sb, NVv[i], z, w, s, p, r, DI[d.dinv_const ? 0 : i], u, mo, acc);
        Z[i] = z; S[i] = s; P[i] = p; R[i] = r; W[i] = w; M[i] = mo;
        if (xp) {
            const T x1 = X[i] + ax * pold;
            X[i] = x1 + sa * p;
        }
    }
    block_sum<kVmaThreads, NV>(acc, lds);
    if (threadIdx.x == 0) {
        double *out = d.part + ((size_t)d.ntiles + wi.tile) * kPartStride;  // slot 1
#pragma unroll
        for (int k = 0; k < NV; ++k)
            out[k] = acc[k];
    }
}

// ---------------------------------------------------------------------------
// SpMV row kernels.

#ifndef PPCG_SPMV_NT
#define PPCG_SPMV_NT 1
#endif

// Matrix entries are read exactly once per SpMV: load them with the
// non-temporal hint so they do not evict the reused input-vector lines.
template <typename T>
__device__ __forceinline__ T stream_load(const PPCG_AS1 T *p)
{
#if PPCG_SPMV_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Value of the stored SELL entry at offset o from the lane's first slot: the
// value itself, or (VI, FP64 values) the entry of the value table `tab` (in
// LDS) named by its one-byte index.  The table holds the matrix's distinct
// values exactly, so both give the same number.
template <bool VI, typename VT>
__device__ __forceinline__ VT sell_value(const PPCG_AS1 VT *v, const PPCG_AS1 unsigned char *vi, const double *tab,
                                         size_t o)
{
    if constexpr (VI)
        return (VT)tab[stream_load(vi + o)];
    else
        return stream_load(v + o);
}

// First stored slot and padded length of a SELL chunk.  A chunk is one
// wavefront's rows, so `chunk` is the same in every lane: taking it from the
// first lane puts both values in scalar registers and makes every guard on
// the chunk length a uniform branch.
__device__ __forceinline__ void sell_extent(const int64_t *__restrict__ cptr, int chunk, int64_t &base, int &len)
{
    const int c = __builtin_amdgcn_readfirstlane(chunk);
    base = as_global(cptr)[c];
    len = (int)((as_global(cptr)[c + 1] - base) / kSellC);
}

// One SpMV input entry x[col].  SC = 1, 2: the input is the preconditioned
// vector m = M^-1 w formed on the fly from w, m[col] = dinv[col] * w[col]
// with the same rounded product the update uses to form m (SC = 1: every
// diagonal entry equal, d0; SC = 2: dinv gathered at dg[col]), so the
// single-launch iteration need not store m.
template <int SC, typename T>
__device__ __forceinline__ T sell_in(const PPCG_AS1 T *x, int col, const double *dg, double d0)
{
    if constexpr (SC == 1)
        return (T)d0 * x[col];
    else if constexpr (SC == 2)
        return (T)as_global(dg)[col] * x[col];
    else
        return x[col];
}

// Entries k0 .. k0 + L - 1 of one SELL row, L fixed at compile time: the
// column and value loads of all L entries are issued back to back, with no
// branch between them, then the L gathers, then the L products are added in
// entry order.  (Guarding each entry by the row length instead puts every
// load in a basic block of its own, and the compiler then waits after each
// one-byte value index or 16-bit column before issuing the next entry.)
// C16: columns as 16-bit offsets from the row, entries 2t and 2t + 1 in one
// dword (pair t at cp[t * 64]); a chunk of odd padded length keeps its last
// entry as one short at `odd`.
template <int L, bool C16, bool VI, int SC, typename VT, typename T, int NX>
__device__ __forceinline__ void sell_span(const PPCG_AS1 int *c, const PPCG_AS1 unsigned *cp,
                                          const PPCG_AS1 short *odd, const PPCG_AS1 VT *v,
                                          const PPCG_AS1 unsigned char *vi, const double *tab,
                                          const PPCG_AS1 T *const (&xg)[NX], int k0, int row, T (&acc)[NX],
                                          const double *dg, double d0)
{
    int cc[L];
    VT vv[L];
    // one base address per stream for the span, the entries at constant
    // offsets from it (immediate offsets of the load instructions, instead of
    // a 64-bit address register per entry)
    const size_t o0 = (size_t)k0 * kSellC;
    if constexpr (C16) {
        const PPCG_AS1 unsigned *cpk = cp + o0 / 2;
#pragma unroll
        for (int t = 0; t < L / 2; ++t) {
            const unsigned pr = stream_load(cpk + t * kSellC);
            cc[2 * t] = row + (int)(short)(pr & 0xffffu);
            cc[2 * t + 1] = row + ((int)pr >> 16);
        }
        if constexpr ((L & 1) != 0)
            cc[L - 1] = row + (int)stream_load(odd);
    } else {
        const PPCG_AS1 int *ck = c + o0;
#pragma unroll
        for (int j = 0; j < L; ++j)
            cc[j] = stream_load(ck + j * kSellC);
    }
    const PPCG_AS1 VT *vk = VI ? nullptr : v + o0;
    const PPCG_AS1 unsigned char *vik = VI ? vi + o0 : nullptr;
#pragma unroll
    for (int j = 0; j < L; ++j)
        vv[j] = sell_value<VI>(vk, vik, tab, (size_t)j * kSellC);
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        T xx[L];
#pragma unroll
        for (int j = 0; j < L; ++j)
            xx[j] = sell_in<SC>(xg[q], cc[j], dg, d0);
#pragma unroll
        for (int j = 0; j < L; ++j)
            acc[q] = acc[q] + (T)vv[j] * xx[j];
    }
}

// The last len - k0 (< M + 1) entries of a row: one uniform compare per
// candidate length, then a straight span of exactly that length.
template <int M, bool C16, bool VI, int SC, typename VT, typename T, int NX>
__device__ __forceinline__ void sell_tail(int rem, const PPCG_AS1 int *c, const PPCG_AS1 unsigned *cp,
                                          const PPCG_AS1 short *odd, const PPCG_AS1 VT *v,
                                          const PPCG_AS1 unsigned char *vi, const double *tab,
                                          const PPCG_AS1 T *const (&xg)[NX], int k0, int row, T (&acc)[NX],
                                          const double *dg, double d0)
{
    if constexpr (M > 0) {
        if (rem == M)
            sell_span<M, C16, VI, SC>(c, cp, odd, v, vi, tab, xg, k0, row, acc, dg, d0);
        else
            sell_tail<M - 1, C16, VI, SC>(rem, c, cp, odd, v, vi, tab, xg, k0, row, acc, dg, d0);
    }
}

// One SELL row (n = A x for NX vectors x): full spans of PPCG_SELL_BATCH
// entries, then the remainder as one span of its exact length.  The row
// length is the same in every lane of the wavefront, so every branch here is
// uniform.  Same products, added in the same (stored) order, as the guarded
// batch loop below.
template <bool C16, bool VI, int SC, typename VT, typename T, int NX>
__device__ __forceinline__ void sell_row_straight(const int64_t *__restrict__ cptr, const int *__restrict__ col,
                                                  const short *__restrict__ col16, const VT *__restrict__ val,
                                                  const T *const (&xin)[NX], int chunk, int lane, T (&acc)[NX],
                                                  const unsigned char *__restrict__ vidx, const double *tab,
                                                  const double *dg, double d0, int64_t ebase = -1, int elen = 0)
{
    constexpr int B = PPCG_SELL_BATCH;
    static_assert(B % 2 == 0, "spans of the 16-bit layout hold whole pairs");
    int64_t base;
    int len;
    if (ebase >= 0) {  // the chunk's extent, loaded by the caller
        base = ebase;
        len = elen;
    } else {
        sell_extent(cptr, chunk, base, len);
    }
    const int row = chunk * kSellC + lane;
    const PPCG_AS1 int *c = C16 ? nullptr : as_global(col + base + lane);
    const PPCG_AS1 unsigned *cp = C16 ? as_global((const unsigned *)(col16 + base) + lane) : nullptr;
    const PPCG_AS1 short *odd = C16 ? as_global(col16 + base + (size_t)(len & ~1) * kSellC + lane) : nullptr;
    const PPCG_AS1 VT *v = VI ? nullptr : as_global(val + base + lane);
    const PPCG_AS1 unsigned char *vi = VI ? as_global(vidx + base + lane) : nullptr;
    const PPCG_AS1 T *xg[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        acc[q] = (T)0;
        xg[q] = as_global(xin[q]);
    }
    int k0 = 0;
    for (; k0 + B <= len; k0 += B)
        sell_span<B, C16, VI, SC>(c, cp, odd, v, vi, tab, xg, k0, row, acc, dg, d0);
    sell_tail<B - 1, C16, VI, SC>(len - k0, c, cp, odd, v, vi, tab, xg, k0, row, acc, dg, d0);
}

// Chunk-shared offset lists.  They are written before any solver launch and
// never during one, and the list of a chunk is the same for its 64 lanes:
// read through the constant address space, so that the uniform loads become
// scalar loads (the few distinct lists stay in the scalar cache) and the
// gathers wait on no vector load.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_constant(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// Entries k0 .. k0 + L - 1 of a row stored on its chunk's shared offset list
// `po`: the column of entry j is row + po[k0 + j], clamped into [0, last]
// (an entry the row lacks is a zero value, at a column that may lie past the
// matrix near its first and last rows).  Then as sell_span: the value loads,
// the gathers, the products added in entry order.
template <int L, bool VI, int SC, typename VT, typename T, int NX>
__device__ __forceinline__ void sell_span_sh(const __attribute__((address_space(4))) int *po,
                                             const PPCG_AS1 VT *v, const PPCG_AS1 unsigned char *vi,
                                             const double *tab, const PPCG_AS1 T *const (&xg)[NX], int k0, int row,
                                             int last, T (&acc)[NX], const double *dg, double d0)
{
    int cc[L];
    VT vv[L];
    const size_t o0 = (size_t)k0 * kSellC;
#pragma unroll
    for (int j = 0; j < L; ++j)
        cc[j] = min(max(row + po[k0 + j], 0), last);
    const PPCG_AS1 VT *vk = VI ? nullptr : v + o0;
    const PPCG_AS1 unsigned char *vik = VI ? vi + o0 : nullptr;
#pragma unroll
    for (int j = 0; j < L; ++j)
        vv[j] = sell_value<VI>(vk, vik, tab, (size_t)j * kSellC);
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        T xx[L];
#pragma unroll
        for (int j = 0; j < L; ++j)
            xx[j] = sell_in<SC>(xg[q], cc[j], dg, d0);
#pragma unroll
        for (int j = 0; j < L; ++j)
            acc[q] = acc[q] + (T)vv[j] * xx[j];
    }
}

// The same span for a chunk whose every column row + po[k] lies inside the
// matrix (all chunks but a few at its first and last rows): no clamp; xr[q]
// points at row's element of input q (and dr at dg's), and each gather
// reads xr[q][po[k]].
template <int L, bool VI, int SC, typename VT, typename T, int NX>
__device__ __forceinline__ void sell_span_in(const __attribute__((address_space(4))) int *po,
                                             const PPCG_AS1 VT *v, const PPCG_AS1 unsigned char *vi,
                                             const double *tab, const PPCG_AS1 T *const (&xr)[NX], int k0,
                                             T (&acc)[NX], const PPCG_AS1 double *dr, double d0)
{
    int oo[L];
    VT vv[L];
    const size_t o0 = (size_t)k0 * kSellC;
#pragma unroll
    for (int j = 0; j < L; ++j)
        oo[j] = po[k0 + j];
    const PPCG_AS1 VT *vk = VI ? nullptr : v + o0;
    const PPCG_AS1 unsigned char *vik = VI ? vi + o0 : nullptr;
#pragma unroll
    for (int j = 0; j < L; ++j)
        vv[j] = sell_value<VI>(vk, vik, tab, (size_t)j * kSellC);
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        T xx[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const T xv = xr[q][oo[j]];
            if constexpr (SC == 1)
                xx[j] = (T)d0 * xv;
            else if constexpr (SC == 2)
                xx[j] = (T)dr[oo[j]] * xv;
            else
                xx[j] = xv;
        }
#pragma unroll
        for (int j = 0; j < L; ++j)
            acc[q] = acc[q] + (T)vv[j] * xx[j];
    }
}

// The last rem (< M + 1) entries of a row on a shared list; IN: the chunk's
// columns all lie inside the matrix (sell_span_in), else sell_span_sh.
// (IN: xg holds the row pointers of sell_span_in, dr its pointer into dg.)
template <int M, bool IN, bool VI, int SC, typename VT, typename T, int NX>
__device__ __forceinline__ void sell_tail_sh(int rem, const __attribute__((address_space(4))) int *po,
                                             const PPCG_AS1 VT *v, const PPCG_AS1 unsigned char *vi,
                                             const double *tab, const PPCG_AS1 T *const (&xg)[NX], int k0, int row,
                                             int last, T (&acc)[NX], const double *dg, const PPCG_AS1 double *dr,
                                             double d0)
{
    if constexpr (M > 0) {
        if (rem == M) {
            if constexpr (IN)
                sell_span_in<M, VI, SC>(po, v, vi, tab, xg, k0, acc, dr, d0);
            else
                sell_span_sh<M, VI, SC>(po, v, vi, tab, xg, k0, row, last, acc, dg, d0);
        } else {
            sell_tail_sh<M - 1, IN, VI, SC>(rem, po, v, vi, tab, xg, k0, row, last, acc, dg, dr, d0);
        }
    }
}

// One SELL row on its chunk's shared offset list (cpat[chunk]: the list's
// start in pats), in straight spans like sell_row_straight.  ebase, elen,
// epat: the chunk's extent and list start, when the caller loaded them.
template <typename VT, typename T, int NX, bool VI = false, int SC = 0>
__device__ __forceinline__ void sell_row_shared(const int64_t *__restrict__ cptr, const int *__restrict__ cpat,
                                                const int *__restrict__ pats, const VT *__restrict__ val,
                                                const T *const (&xin)[NX], int chunk, int lane, int n, T (&acc)[NX],
                                                const unsigned char *__restrict__ vidx = nullptr,
                                                const double *tab = nullptr, const double *dg = nullptr,
                                                double d0 = 0.0, int64_t ebase = -1, int elen = 0, int epat = -1)
{
    constexpr int B = PPCG_SHARED_BATCH;
    int64_t base;
    int len;
    if (ebase >= 0) {
        base = ebase;
        len = elen;
    } else {
        sell_extent(cptr, chunk, base, len);
    }
    const int ps = epat >= 0 ? epat : as_constant(cpat)[__builtin_amdgcn_readfirstlane(chunk)];
    const __attribute__((address_space(4))) int *po = as_constant(pats) + ps;
    const int row = chunk * kSellC + lane;
    const PPCG_AS1 VT *v = VI ? nullptr : as_global(val + base + lane);
    const PPCG_AS1 unsigned char *vi = VI ? as_global(vidx + base + lane) : nullptr;
    const PPCG_AS1 T *xg[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        acc[q] = (T)0;
        xg[q] = as_global(xin[q]);
    }
    if (len < 1)
        return;
    // the list ascends: its first and last offsets bound the chunk's columns
    const int c0 = chunk * kSellC;
    const bool inside = c0 + po[0] >= 0 && (int64_t)c0 + (kSellC - 1) + po[len - 1] < (int64_t)n;
    int k0 = 0;
    if (inside) {
        const PPCG_AS1 T *xr[NX];
#pragma unroll
        for (int q = 0; q < NX; ++q)
            xr[q] = xg[q] + row;
        const PPCG_AS1 double *dr = SC == 2 ? as_global(dg) + row : nullptr;
        for (; k0 + B <= len; k0 += B)
            sell_span_in<B, VI, SC>(po, v, vi, tab, xr, k0, acc, dr, d0);
        sell_tail_sh<B - 1, true, VI, SC>(len - k0, po, v, vi, tab, xr, k0, row, n - 1, acc, dg, dr, d0);
    } else {
        for (; k0 + B <= len; k0 += B)
            sell_span_sh<B, VI, SC>(po, v, vi, tab, xg, k0, row, n - 1, acc, dg, d0);
        sell_tail_sh<B - 1, false, VI, SC>(len - k0, po, v, vi, tab, xg, k0, row, n - 1, acc, dg, nullptr, d0);
    }
}

// SELL-C-sigma, C = 64, one lane per row: entry k of the row (chunk c, lane
// l) is at cptr[c] + k * 64 + l.  NX input vectors share one pass over the
// matrix (NX = 2 for the replacement steps).  Entries are handled in
// batches of 8: the column indices and values of a batch are loaded first,
// then its gathers are issued, so each lane has up to 16 independent loads
// in flight; the products of every row are still added in stored
// (ascending original column) order.  VT is the value type, T the vector
// and accumulation type.
template <typename VT, typename T, int NX, bool VI = false, int SC = 0>
__device__ __forceinline__ void sell_row(const int64_t *__restrict__ cptr, const int *__restrict__ col,
                                         const VT *__restrict__ val, const T *const (&xin)[NX], int chunk,
                                         int lane, T (&acc)[NX], const unsigned char *__restrict__ vidx = nullptr,
                                         const double *tab = nullptr, const double *dg = nullptr, double d0 = 0.0,
                                         int64_t ebase = -1, int elen = 0)
{
#if PPCG_SELL_STRAIGHT
    // (32-bit columns with 8-byte values measured 2-3 % faster in the guarded
    // loop below: their loads already issue back to back there)
    if constexpr (VI || (SC != 0 && PPCG_SELL_STRAIGHT_SC))
        return sell_row_straight<false, VI, SC, VT, T, NX>(cptr, col, nullptr, val, xin, chunk, lane, acc, vidx, tab,
                                                           dg, d0, ebase, elen);
#endif
    constexpr int B = PPCG_SELL_BATCH;
    int64_t base;
    int len;
    if (ebase >= 0) {  // the chunk's extent, loaded by the caller
        base = ebase;
        len = elen;
    } else {
        sell_extent(cptr, chunk, base, len);
    }
    const PPCG_AS1 int *c = as_global(col + base + lane);
    const PPCG_AS1 VT *v = VI ? nullptr : as_global(val + base + lane);
    const PPCG_AS1 unsigned char *vi = VI ? as_global(vidx + base + lane) : nullptr;
    const PPCG_AS1 T *xg[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        acc[q] = (T)0;
        xg[q] = as_global(xin[q]);
    }
    for (int k0 = 0; k0 < len; k0 += B) {
        int cc[B];
        VT vv[B];
        // len is the same for every lane of the wavefront (one chunk), so
        // these guards are uniform branches, not divergence.
#pragma unroll
        for (int j = 0; j < B; ++j) {
            cc[j] = 0;
            vv[j] = (VT)0;
            if (k0 + j < len) {
                cc[j] = stream_load(c + (size_t)(k0 + j) * kSellC);
                vv[j] = sell_value<VI>(v, vi, tab, (size_t)(k0 + j) * kSellC);
            }
        }
#pragma unroll
        for (int q = 0; q < NX; ++q) {
            T xx[B];
#pragma unroll
            for (int j = 0; j < B; ++j)
                xx[j] = k0 + j < len ? sell_in<SC>(xg[q], cc[j], dg, d0) : (T)0;
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (k0 + j < len)
                    acc[q] = acc[q] + (T)vv[j] * xx[j];
        }
    }
}

// Column indices of entries k0 .. k0 + B - 1 of one SELL row from 16-bit
// offsets stored in pairs (see k_sell_delta16): entries 2j and 2j + 1 of the
// lane come in one dword, the last entry of an odd-length chunk as one short.
// base: the chunk's first slot, len: its padded length (uniform over the
// wavefront, so the guards are uniform branches), row: the stored row.
// Entries past len get the row itself (a valid index, never used).
template <int B>
__device__ __forceinline__ void sell_cols16(const short *__restrict__ col16, int64_t base, int len, int k0, int lane,
                                            int row, int (&cc)[B])
{
    static_assert(B % 2 == 0, "batches hold whole pairs");
    const int paired = len & ~1;
    const PPCG_AS1 unsigned *cp = as_global((const unsigned *)(col16 + base) + lane);  // pair j at cp[j * 64]
#pragma unroll
    for (int t = 0; t < B / 2; ++t) {
        const int k = k0 + 2 * t;
        cc[2 * t] = row;
        cc[2 * t + 1] = row;
        if (k + 1 < len) {
            const unsigned pr = stream_load(cp + (size_t)(k >> 1) * kSellC);
            cc[2 * t] = row + (int)(short)(pr & 0xffffu);
            cc[2 * t + 1] = row + ((int)pr >> 16);
        } else if (k < len) {
            cc[2 * t] = row + (int)stream_load(as_global(col16 + base + (size_t)paired * kSellC + lane));
        }
    }
}

// sell_row with 16-bit column offsets from the row.
template <typename VT, typename T, int NX, bool VI = false, int SC = 0>
__device__ __forceinline__ void sell_row16(const int64_t *__restrict__ cptr, const short *__restrict__ col16,
                                           const VT *__restrict__ val, const T *const (&xin)[NX], int chunk,
                                           int lane, T (&acc)[NX], const unsigned char *__restrict__ vidx = nullptr,
                                           const double *tab = nullptr, const double *dg = nullptr, double d0 = 0.0,
                                           int64_t ebase = -1, int elen = 0)
{
#if PPCG_SELL_STRAIGHT
    return sell_row_straight<true, VI, SC, VT, T, NX>(cptr, nullptr, col16, val, xin, chunk, lane, acc, vidx, tab,
                                                      dg, d0, ebase, elen);
#endif
    constexpr int B = PPCG_SELL_BATCH;
    int64_t base;
    int len;
    if (ebase >= 0) {  // the chunk's extent, loaded by the caller
        base = ebase;
        len = elen;
    } else {
        sell_extent(cptr, chunk, base, len);
    }
    const int row = chunk * kSellC + lane;
    const PPCG_AS1 VT *v = VI ? nullptr : as_global(val + base + lane);
    const PPCG_AS1 unsigned char *vi = VI ? as_global(vidx + base + lane) : nullptr;
    const PPCG_AS1 T *xg[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        acc[q] = (T)0;
        xg[q] = as_global(xin[q]);
    }
    for (int k0 = 0; k0 < len; k0 += B) {
        int cc[B];
        VT vv[B];
        sell_cols16<B>(col16, base, len, k0, lane, row, cc);
#pragma unroll
        for (int j = 0; j < B; ++j) {
            vv[j] = (VT)0;
            if (k0 + j < len)
                vv[j] = sell_value<VI>(v, vi, tab, (size_t)(k0 + j) * kSellC);
        }
#pragma unroll
        for (int q = 0; q < NX; ++q) {
            T xx[B];
#pragma unroll
            for (int j = 0; j < B; ++j)
                xx[j] = k0 + j < len ? sell_in<SC>(xg[q], cc[j], dg, d0) : (T)0;
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (k0 + j < len)
                    acc[q] = acc[q] + (T)vv[j] * xx[j];
        }
    }
}

// sell_row16 software-pipelined across batches: the gathers of batch k are
// issued before the column and value loads of batch k + 1, so the wait for
// the gathers leaves the next batch's loads in flight.  Same products, same
// order of the sums.
template <typename VT, typename T, int NX, bool VI = false, int SC = 0>
__device__ __forceinline__ void sell_row16_pipe(const int64_t *__restrict__ cptr, const short *__restrict__ col16,
                                                const VT *__restrict__ val, const T *const (&xin)[NX], int chunk,
                                                int lane, T (&acc)[NX],
                                                const unsigned char *__restrict__ vidx = nullptr,
                                                const double *tab = nullptr, const double *dg = nullptr,
                                                double d0 = 0.0, int64_t ebase = -1, int elen = 0)
{
#if PPCG_SELL_STRAIGHT
    return sell_row_straight<true, VI, SC, VT, T, NX>(cptr, nullptr, col16, val, xin, chunk, lane, acc, vidx, tab,
                                                      dg, d0, ebase, elen);
#endif
    constexpr int B = PPCG_SELL_PIPE_BATCH;  // two batches in flight: smaller than the plain batch
    int64_t base;
    int len;
    if (ebase >= 0) {  // the chunk's extent, loaded by the caller
        base = ebase;
        len = elen;
    } else {
        sell_extent(cptr, chunk, base, len);
    }
    const int row = chunk * kSellC + lane;
    const PPCG_AS1 VT *v = VI ? nullptr : as_global(val + base + lane);
    const PPCG_AS1 unsigned char *vi = VI ? as_global(vidx + base + lane) : nullptr;
    const PPCG_AS1 T *xg[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        acc[q] = (T)0;
        xg[q] = as_global(xin[q]);
    }
    int cc[B];
    VT vv[B];
    auto load_batch = [&](int k0, int (&c)[B], VT (&w)[B]) {
        sell_cols16<B>(col16, base, len, k0, lane, row, c);
#pragma unroll
        for (int j = 0; j < B; ++j) {
            w[j] = (VT)0;
            if (k0 + j < len)
                w[j] = sell_value<VI>(v, vi, tab, (size_t)(k0 + j) * kSellC);
        }
    };
    if (len > 0)
        load_batch(0, cc, vv);
    for (int k0 = 0; k0 < len; k0 += B) {
        T xx[NX][B];
#pragma unroll
        for (int q = 0; q < NX; ++q)
#pragma unroll
            for (int j = 0; j < B; ++j)
                xx[q][j] = k0 + j < len ? sell_in<SC>(xg[q], cc[j], dg, d0) : (T)0;
        int cn[B];
        VT vn[B];
        if (k0 + B < len)
            load_batch(k0 + B, cn, vn);
#pragma unroll
        for (int q = 0; q < NX; ++q)
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (k0 + j < len)
                    acc[q] = acc[q] + (T)vv[j] * xx[q][j];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            cc[j] = cn[j];
            vv[j] = vn[j];
        }
    }
}

// CSR-vector: a group of L lanes per row (L a power of two in [2, 64]); lane
// k of the group sums entries k, k + L, ... and the group combines its lanes
// with a butterfly.  Result valid in every lane of the group.
template <typename VT, typename T, int NX>
__device__ __forceinline__ void csrv_row(const int *__restrict__ rp, const int *__restrict__ col,
                                         const VT *__restrict__ val, const T *const (&xin)[NX], int i, int n, int L,
                                         int l, T (&acc)[NX])
{
#pragma unroll
    for (int q = 0; q < NX; ++q)
        acc[q] = (T)0;
    if (i < n) {
        const int e = as_global(rp)[i + 1];
        for (int k = as_global(rp)[i] + l; k < e; k += L) {
            const T a = (T)stream_load(as_global(val + k));
            const int cc = stream_load(as_global(col + k));
#pragma unroll
            for (int q = 0; q < NX; ++q)
                acc[q] = acc[q] + a * as_global(xin[q])[cc];
        }
    }
#pragma unroll
    for (int q = 0; q < NX; ++q)
        for (int off = L >> 1; off >= 1; off >>= 1)
            acc[q] = acc[q] + __shfl_xor(acc[q], off, 64);
}

// Inputs of each mode.
template <int MODE> struct SpmvIn { static constexpr int NX = 1; };
template <> struct SpmvIn<MODE_DUAL1> { static constexpr int NX = 2; };
template <> struct SpmvIn<MODE_DUAL2> { static constexpr int NX = 2; };

template <typename T, int MODE>
__device__ __forceinline__ void spmv_inputs(const SysDesc &d, const T *(&x)[SpmvIn<MODE>::NX])
{
    if constexpr (MODE == MODE_ITER) {
        x[0] = (const T *)d.m;
    } else if constexpr (MODE == MODE_INIT2) {
        x[0] = (const T *)d.u;
    } else if constexpr (MODE == MODE_DUAL1) {
        x[0] = (const T *)d.u;
        x[1] = (const T *)d.p;
    } else if constexpr (MODE == MODE_DUAL2) {
        x[0] = (const T *)d.m;
        x[1] = (const T *)d.q;
    } else {  // INIT1, RESID, PLAIN, REPL1
        x[0] = (const T *)d.x;
    }
}

// Modes that form a true residual b - A x always use the FP64 values; the
// iteration's own products use the FP32 copy in vals32 mode.
template <int MODE> constexpr bool kTrueOperator =
    MODE == MODE_INIT1 || MODE == MODE_INIT0 || MODE == MODE_RESID || MODE == MODE_REPL1;

// Per-row epilogue of each mode; accumulates this row's share of the partials.
template <typename T, int MODE>
__device__ __forceinline__ void spmv_epilogue(const SysDesc &d, int i, const T (&y)[SpmvIn<MODE>::NX],
                                              double (&acc)[kReplPartials])
{
    const PPCG_AS1 T *DI = as_global((const T *)d.dinv);
    if constexpr (MODE == MODE_ITER || MODE == MODE_PLAIN) {
        as_global((T *)d.nv)[i] = y[0];
    } else if constexpr (MODE == MODE_INIT1 || MODE == MODE_INIT0 || MODE == MODE_REPL1) {
        const T bi = as_global((const T *)d.b)[i];
        const T ri = bi - y[0];
        const T ui = DI[i] * ri;
        as_global((T *)d.r)[i] = ri;
        as_global((T *)d.u)[i] = ui;
        if constexpr (MODE == MODE_INIT1 || MODE == MODE_INIT0) {
            // z, q, s, p enter the first update multiplied by beta = 0: start
            // them at zero so that stale memory (possibly NaN) cannot leak in.
            as_global((T *)d.z)[i] = (T)0;
            as_global((T *)d.q)[i] = (T)0;
            as_global((T *)d.s)[i] = (T)0;
            as_global((T *)d.p)[i] = (T)0;
        }
        acc[0] = acc[0] + (double)bi * (double)bi;
    } else if constexpr (MODE == MODE_INIT2) {
        const T ri = as_global((const T *)d.r)[i];
        const T ui = as_global((const T *)d.u)[i];
        const T mi = DI[i] * y[0];
        as_global((T *)d.w)[i] = y[0];
        as_global((T *)d.m)[i] = mi;
        const double rd = (double)ri, ud = (double)ui, wd = (double)y[0];
        acc[0] = acc[0] + rd * ud;
        acc[1] = acc[1] + wd * ud;
        acc[2] = acc[2] + ud * ud;
        acc[3] = acc[3] + rd * rd;
    } else if constexpr (MODE == MODE_DUAL1) {
        const T ri = as_global((const T *)d.r)[i];
        const T ui = as_global((const T *)d.u)[i];
        const T pi = as_global((const T *)d.p)[i];
        as_global((T *)d.w)[i] = y[0];
        as_global((T *)d.s)[i] = y[1];
        as_global((T *)d.m)[i] = DI[i] * y[0];
        as_global((T *)d.q)[i] = DI[i] * y[1];
        const double rd = (double)ri, ud = (double)ui, wd = (double)y[0], sd = (double)y[1], pd = (double)pi;
        acc[0] = acc[0] + rd * ud;
        acc[1] = acc[1] + wd * ud;
        acc[2] = acc[2] + ud * ud;
        acc[3] = acc[3] + rd * rd;
        acc[4] = acc[4] + ud * sd;
        acc[5] = acc[5] + pd * sd;
    } else if constexpr (MODE == MODE_DUAL2) {
        as_global((T *)d.nv)[i] = y[0];
        as_global((T *)d.z)[i] = y[1];
    } else if constexpr (MODE == MODE_RESID) {
        const T bi = as_global((const T *)d.b)[i];
        const T ti = bi - y[0];
        as_global((T *)d.r)[i] = ti;
        acc[0] = acc[0] + (double)ti * (double)ti;
        acc[1] = acc[1] + (double)bi * (double)bi;
    }
}

// Work of the designated workgroup of a system after its SpMV tile: reduce
// the partials of the previous launch and update the scalars.  Kept out of
// line so that its registers do not add to the SpMV's register pressure.
template <int MODE>
__device__ __noinline__ void designated_reduce(const SysDesc &d, SysState *st, double *lds)
{
    // After a fused update (not the ITER pass that ends the initialisation):
    // it either deferred its x-update (alpha of this iteration kept) or
    // applied the deferred one with its own.
    auto note_x = [&]() {
        if (!st->phase) {
            st->alpha_x = st->alpha;
            st->x_pending ^= 1;
        }
    };
    if constexpr (MODE == MODE_DUAL2) {
        double v[kReplPartials];
        reduce_partials<kSpmvThreads, kReplPartials>(d, 1, v, lds);
        if (threadIdx.x == 0)
            scalar_update_repl(d, st, v);
    } else if (MODE == MODE_ITER && d.vals32) {
        double v[kReplPartials];
        reduce_partials<kSpmvThreads, kReplPartials>(d, 1, v, lds);
        if (threadIdx.x == 0) {
            note_x();
            scalar_update<kReplPartials>(d, st, v);
        }
    } else {
        double v[kNumPartials];
        reduce_partials<kSpmvThreads>(d, MODE == MODE_INIT2 ? 0 : 1, v, lds);
        if (threadIdx.x == 0) {
            if (MODE == MODE_INIT2) {
                st->bnorm2 = v[0];
            } else {
                note_x();
                scalar_update<kNumPartials>(d, st, v);
            }
        }
    }
}

// tab: the system's value table in LDS when it reads one-byte value indices
// (FP64 values only), else NULL.
template <typename VT, typename T, int MODE>
__device__ __forceinline__ void spmv_tile(const SysDesc &d, const VT *__restrict__ val, const WorkItem wi,
                                          double (&acc)[kReplPartials], const double *tab = nullptr)
{
    constexpr int NX = SpmvIn<MODE>::NX;
    const T *xin[NX];
    spmv_inputs<T, MODE>(d, xin);
    const int n = d.n;
    T y[NX];
    if constexpr (MODE == MODE_INIT0) {
        // A x with x = 0 is +0 in every row: the epilogues run on the rows
        // and in the order of the format's SpMV (the same partial sums)
        y[0] = (T)0;
        if (d.fmt == FMT_SELL) {
            const int chunk = wi.tile * kSellChunksPerTile + (threadIdx.x >> 6);
            const int i = chunk * kSellC + (threadIdx.x & 63);
            if (chunk * kSellC < n && i < n)
                spmv_epilogue<T, MODE>(d, i, y, acc);
        } else {
            const int L = d.lanes;
            const int g = threadIdx.x / L, l = threadIdx.x % L;
            const int rows_per_pass = kSpmvThreads / L;
            for (int pass = 0; pass < kTileRows / rows_per_pass; ++pass) {
                const int i = wi.tile * kTileRows + pass * rows_per_pass + g;
                if (l == 0 && i < n)
                    spmv_epilogue<T, MODE>(d, i, y, acc);
            }
        }
        return;
    }
    if (d.fmt == FMT_SELL) {
        static_assert(kTileRows == kSpmvThreads, "SELL path: one row per lane");
        const int lane = threadIdx.x & 63;
        const int chunk = wi.tile * kSellChunksPerTile + (threadIdx.x >> 6);
        const int i = chunk * kSellC + lane;
        if (chunk * kSellC < n) {
            // both choices are uniform per system
            bool done = false;
            // shared offset lists: FP64 vectors, FP64 values (with or
            // without the value table) or FP32 values
            if constexpr (std::is_same<T, double>::value && NX == 1) {
                if (d.cpat) {
                    if constexpr (std::is_same<VT, double>::value) {
                        if (tab)
                            sell_row_shared<VT, T, NX, true>(d.cptr, d.cpat, d.pats, val, xin, chunk, lane, n, y,
                                                             d.vidx, tab);
                        else
                            sell_row_shared<VT, T, NX>(d.cptr, d.cpat, d.pats, val, xin, chunk, lane, n, y);
                    } else {
                        sell_row_shared<VT, T, NX>(d.cptr, d.cpat, d.pats, val, xin, chunk, lane, n, y);
                    }
                    done = true;
                }
            }
            if constexpr (std::is_same<VT, double>::value && NX == 1) {
                if (!done && tab) {
                    if (d.col16)
#if PPCG_SELL_PIPE
                        sell_row16_pipe<VT, T, NX, true>(d.cptr, d.col16, val, xin, chunk, lane, y, d.vidx, tab);
#else
                        sell_row16<VT, T, NX, true>(d.cptr, d.col16, val, xin, chunk, lane, y, d.vidx, tab);
#endif
                    else
                        sell_row<VT, T, NX, true>(d.cptr, d.col, val, xin, chunk, lane, y, d.vidx, tab);
                    done = true;
                }
            }
            if (!done) {
                if (d.col16)
#if PPCG_SELL_PIPE
                    sell_row16_pipe<VT, T, NX>(d.cptr, d.col16, val, xin, chunk, lane, y);
#else
                    sell_row16<VT, T, NX>(d.cptr, d.col16, val, xin, chunk, lane, y);
#endif
                else
                    sell_row<VT, T, NX>(d.cptr, d.col, val, xin, chunk, lane, y);
            }
            if (i < n)
                spmv_epilogue<T, MODE>(d, i, y, acc);
        }
    } else {
        const int L = d.lanes;
        const int g = threadIdx.x / L, l = threadIdx.x % L;
        const int rows_per_pass = kSpmvThreads / L;
        const int passes = kTileRows / rows_per_pass;
        for (int pass = 0; pass < passes; ++pass) {
            const int i = wi.tile * kTileRows + pass * rows_per_pass + g;
            csrv_row<VT, T, NX>(d.rp, d.col, val, xin, i, n, L, l, y);
            if (l == 0 && i < n)
                spmv_epilogue<T, MODE>(d, i, y, acc);
        }
    }
}

// Eight waves per SIMD (at most 64 VGPRs): the gathers depend on the column
// loads, so latency is hidden by the number of waves in flight.
template <typename T, int MODE>
__global__ __launch_bounds__(kSpmvThreads, PPCG_SPMV_WAVES) void k_spmv(const WorkItem *__restrict__ table,
                                                          const int *__restrict__ count,
                                                          const SysDesc *__restrict__ descs, int remap)
{
    __shared__ double lds[kSpmvThreads / 64 * kReplPartials];
    // Graphs bake a grid that may exceed the live table: blocks past it exit,
    // and the XCD-aware order is taken over the live items only, so that
    // every XCD gets an equal share of them.
    const int live = *count;
    if ((int)blockIdx.x >= live)
        return;
    const int pos = remap ? xcd_remap(blockIdx.x, live) : (int)blockIdx.x;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    SysState *st = d.st;
    if (MODE == MODE_ITER && st->done)
        return;
    double acc[kReplPartials] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (!kTrueOperator<MODE> && d.vals32) {
        spmv_tile<float, T, MODE>(d, d.val32, wi, acc);
    } else if (std::is_same<T, double>::value && SpmvIn<MODE>::NX == 1 && d.vidx && d.fmt == FMT_SELL) {
        // the value table, once per workgroup (one work item: uniform); the
        // two-vector SpMVs of the reliable updates read the values
        __shared__ double vtab[kMaxValueTable];
        for (int t = threadIdx.x; t < d.nvtab; t += kSpmvThreads)
            vtab[t] = d.vtab[t];
        __syncthreads();
        spmv_tile<T, T, MODE>(d, (const T *)d.val, wi, acc, vtab);
    } else {
        spmv_tile<T, T, MODE>(d, (const T *)d.val, wi, acc);
    }
    constexpr bool kWritesPartials =
        MODE == MODE_INIT1 || MODE == MODE_INIT0 || MODE == MODE_INIT2 || MODE == MODE_RESID || MODE == MODE_DUAL1;
    if constexpr (kWritesPartials) {
        constexpr int NV = MODE == MODE_DUAL1 ? kReplPartials : kNumPartials;
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k)
            v[k] = acc[k];
        block_sum<kSpmvThreads, NV>(v, lds);
        if (threadIdx.x == 0) {
            const int slot = (MODE == MODE_INIT2 || MODE == MODE_DUAL1) ? 1 : 0;
            double *out = d.part + ((size_t)slot * d.ntiles + wi.tile) * kPartStride;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                out[k] = v[k];
            if constexpr (MODE == MODE_INIT2) {
                out[4] = 0.0;  // the direct-denominator terms are unused at a start
                out[5] = 0.0;
            }
        }
    }
    if (wi.tile != 0)
        return;
    // Designated workgroup of this system.
    if constexpr (MODE == MODE_INIT1 || MODE == MODE_INIT0) {
        if (threadIdx.x == 0) {
            st->phase = 1;
            st->i_start = 0;
            st->done = 0;
            st->status = ST_OK;
            st->x_pending = 0;  // a start reads a complete x (k_x_fixup ran before)
        }
    } else if constexpr (MODE == MODE_INIT2 || MODE == MODE_ITER || MODE == MODE_DUAL2) {
        __syncthreads();  // lds reuse
        designated_reduce<MODE>(d, st, lds);
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

// Deferred x-updates (see vma_elem): for the systems whose last x-update is
// still pending, x += alpha_x p (p is still that iteration's direction).
// Run before anything reads x; k_x_settle then clears the flag, in a launch
// of its own so that no workgroup of this one can see it cleared early.
template <typename T>
__global__ void k_x_fixup(const WorkItem *__restrict__ table, const int *__restrict__ count,
                          const SysDesc *__restrict__ descs)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    const SysState *st = d.st;
    if (!st->x_pending)
        return;
    const T a = (T)st->alpha_x;
    PPCG_AS1 T *__restrict__ X = as_global((T *)d.x);
    const PPCG_AS1 T *__restrict__ P = as_global((const T *)d.p);
    for (int k = threadIdx.x; k < kTileRows; k += blockDim.x) {
        const int i = wi.tile * kTileRows + k;
        if (i < d.n)
            X[i] = X[i] + a * P[i];
    }
}

__global__ void k_x_settle(const WorkItem *__restrict__ table, const int *__restrict__ count,
                           const SysDesc *__restrict__ descs)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    if (wi.tile == 0 && threadIdx.x == 0)
        descs[wi.slot].st->x_pending = 0;
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

// One vector move of a batched solve's staging (perm may be null):
// STAGE_GATHER dst[i] = src[perm[i]], STAGE_ZERO dst[i] = 0,
// STAGE_SCATTER dst[perm[i]] = src[i].
enum StageOp : int { STAGE_GATHER = 0, STAGE_ZERO = 1, STAGE_SCATTER = 2 };
struct StageItem {
    const int *perm;
    const double *src;
    double *dst;
    int n;
    int op;
};

// All moves of a batch in one launch: grid.y strides over the items,
// grid.x (with a grid stride) over each item's rows.
__global__ void k_stage_batch(const StageItem *__restrict__ items, int count)
{
    for (int it = blockIdx.y; it < count; it += gridDim.y) {
        const StageItem s = items[it];
        const int stride = gridDim.x * blockDim.x;
        if (s.op == STAGE_GATHER) {
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride)
                s.dst[i] = s.src[s.perm ? s.perm[i] : i];
        } else if (s.op == STAGE_ZERO) {
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride)
                s.dst[i] = 0.0;
        } else {
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.n; i += stride)
                s.dst[s.perm ? s.perm[i] : i] = s.src[i];
        }
    }
}

}  // namespace ppcg
