// ppcg_pcg.hpp -- classic PCG (Algorithm 1 of Tiwari & Vadhiyar, Section
// III-A) on the device, for comparison with the pipelined method, and as the
// iteration of the FP32-values mode when selected.
//
// One iteration is four launches:
//
//   k_pcg_spmv      (per tile)   p = u + beta p, formed on the fly for every
//                                gathered entry and written for the tile's
//                                own rows into the other buffer of a
//                                double-buffered pair; s = A p; partial sums
//                                of (s, p).
//   k_pcg_alpha     (per system) reduce (s, p) in a fixed order; alpha.
//   k_pcg_vma       (per tile)   x += alpha p, r -= alpha s, u = M^-1 r;
//                                partial sums of (u, r), (u, u), (r, r).
//   k_pcg_update    (per system) reduce them; stopping test; beta.
//
// Unlike Algorithm 2, each of the two reductions gates the next launch, so
// they cannot be hidden behind other work: they run as one-workgroup-per-
// system kernels between the streaming kernels (no grid-wide fences or
// atomics).  Which buffer of the pair holds the current direction follows
// from the iteration counter: the SpMV of the iteration after k x-updates
// reads buffer k mod 2 (p for even, z for odd) and writes the other.
//
// The kernels are templated on the vector type T: double for the FP64 and
// FP32-values modes, float for the FP32 mixed-precision mode (FP32 vectors
// and values, FP64 dot-product accumulation and scalars), which always
// iterates with Algorithm 1.
//
// FP32 mixed-precision mode (d.prec == PREC_F32): one Algorithm 1 sequence
// in FP32 on the scaled system A y = r64 / ||r64||, paused like the
// FP32-values mode below.  At a pause the host adds the correction to the
// FP64 iterate (k_pcg_mix_correct), recomputes r64 = b - A64 x64 and, unless
// it has converged, rescales the system to the new residual
// (k_pcg_mix_start: the kept direction and gamma_{i-1} are carried over to
// the new scale) and replaces r32, u32 as in a reliable update; the Krylov
// sequence continues instead of restarting.
//
// FP32-values mode (d.vals32): s = A32 p with FP32 matrix values, FP64
// vectors and accumulation.  When the recurrence residual has fallen by
// d.repl_factor since the last start or reliable update, the system pauses
// (ST_REPLACE); the host then recomputes r = b - A64 x and u = M^-1 r and the
// iteration continues with the same direction (beta from the replaced
// residual), the residual-replacement scheme for classic CG.
#pragma once

#include "ppcg_kernels.hpp"

namespace ppcg {

// Threads of the one-workgroup-per-system reduction kernels.
constexpr int kPcgRedThreads = 1024;

// FP32 mixed precision with classic PCG: default residual reduction between
// reliable updates (ppcg_options.inner_tol overrides it).
constexpr double kPcgMixReplFactor = 1e-2;

// Fixed-order reduction of NV partials over a system's tiles for the
// one-workgroup reduction kernels: thread t takes the tiles t, t + NT, ...
// in index order, with the loads of kPcgRedBatch tiles issued before their
// sums (one memory latency per batch), then the workgroup tree.
constexpr int kPcgRedBatch = 4;

template <int NV>
__device__ __forceinline__ void pcg_reduce(const SysDesc &d, int slot, double (&out)[NV], double *lds)
{
    const PPCG_AS1 double *P = as_global(d.part + (size_t)slot * d.ntiles * kPartStride);
#pragma unroll
    for (int k = 0; k < NV; ++k)
        out[k] = 0.0;
    for (int t0 = threadIdx.x; t0 < d.ntiles; t0 += kPcgRedBatch * kPcgRedThreads) {
        double v[kPcgRedBatch][NV];
#pragma unroll
        for (int j = 0; j < kPcgRedBatch; ++j) {
            const int t = t0 + j * kPcgRedThreads;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                v[j][k] = t < d.ntiles ? P[(size_t)t * kPartStride + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kPcgRedBatch; ++j)
            if (t0 + j * kPcgRedThreads < d.ntiles) {
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    out[k] = out[k] + v[j][k];
            }
    }
    block_sum<kPcgRedThreads, NV>(out, lds);
}

// Direction buffers: the current direction after k x-updates is in pcg_dir(k).
template <typename T>
__device__ __forceinline__ T *pcg_dir(const SysDesc &d, int k)
{
    return (T *)((k & 1) ? d.z : d.p);
}

// Entries k0 .. k0 + L - 1 of one row of s = A p (L fixed at compile time):
// the column and value loads of all L entries back to back, then the gathers
// of u and p_old, then the products added in entry order (the order of the
// guarded loop below, so the same sums).  Bases at constant offsets per
// entry, as in sell_span.
// CM: the column layout, 0 = 32-bit columns, 1 = 16-bit offsets in pairs,
// 2 = the chunk's shared offset list po (columns row + po[k], clamped into
// [0, last]).
template <int L, int CM, typename T, typename VT>
__device__ __forceinline__ void pcg_span(const PPCG_AS1 int *c, const PPCG_AS1 unsigned *cp,
                                         const PPCG_AS1 short *odd, const __attribute__((address_space(4))) int *po,
                                         int last, const PPCG_AS1 VT *v, int k0, int row, T beta,
                                         const PPCG_AS1 T *__restrict__ U, const PPCG_AS1 T *__restrict__ Pold, T &y)
{
    int cc[L];
    T vv[L], xx[L];
    const size_t o0 = (size_t)k0 * kSellC;
    if constexpr (CM == 2) {
#pragma unroll
        for (int j = 0; j < L; ++j)
            cc[j] = min(max(row + po[k0 + j], 0), last);
    } else if constexpr (CM == 1) {
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
    const PPCG_AS1 VT *vk = v + o0;
#pragma unroll
    for (int j = 0; j < L; ++j)
        vv[j] = (T)stream_load(vk + j * kSellC);
#pragma unroll
    for (int j = 0; j < L; ++j)
        xx[j] = U[cc[j]] + beta * Pold[cc[j]];
#pragma unroll
    for (int j = 0; j < L; ++j)
        y = y + vv[j] * xx[j];
}

template <int M, int CM, typename T, typename VT>
__device__ __forceinline__ void pcg_tail(int rem, const PPCG_AS1 int *c, const PPCG_AS1 unsigned *cp,
                                         const PPCG_AS1 short *odd, const __attribute__((address_space(4))) int *po,
                                         int last, const PPCG_AS1 VT *v, int k0, int row, T beta,
                                         const PPCG_AS1 T *__restrict__ U, const PPCG_AS1 T *__restrict__ Pold, T &y)
{
    if constexpr (M > 0) {
        if (rem == M)
            pcg_span<M, CM>(c, cp, odd, po, last, v, k0, row, beta, U, Pold, y);
        else
            pcg_tail<M - 1, CM>(rem, c, cp, odd, po, last, v, k0, row, beta, U, Pold, y);
    }
}

// One SELL row of s = A p with p = u + beta p_old formed per gathered entry.
// CM: the column layout (pcg_span).  Full spans of 8 entries, then one span
// of the remaining length.
template <int CM, typename T, typename VT>
__device__ __forceinline__ T pcg_sell_row(const SysDesc &d, const VT *__restrict__ val, int chunk, int lane,
                                          T beta, const PPCG_AS1 T *__restrict__ U,
                                          const PPCG_AS1 T *__restrict__ Pold)
{
    constexpr bool C16 = CM == 1;
#if PPCG_SELL_STRAIGHT
    {
        constexpr int B = 8;
        int64_t base;
        int len;
        sell_extent(d.cptr, chunk, base, len);
        const int row = chunk * kSellC + lane;
        const PPCG_AS1 int *c = CM == 0 ? as_global(d.col + base + lane) : nullptr;
        const PPCG_AS1 unsigned *cp = C16 ? as_global((const unsigned *)(d.col16 + base) + lane) : nullptr;
        const PPCG_AS1 short *odd = C16 ? as_global(d.col16 + base + (size_t)(len & ~1) * kSellC + lane) : nullptr;
        const __attribute__((address_space(4))) int *po = nullptr;
        if constexpr (CM == 2)
            po = as_constant(d.pats) + as_constant(d.cpat)[__builtin_amdgcn_readfirstlane(chunk)];
        const PPCG_AS1 VT *v = as_global(val + base + lane);
        T y = 0;
        int k0 = 0;
        for (; k0 + B <= len; k0 += B)
            pcg_span<B, CM>(c, cp, odd, po, d.n - 1, v, k0, row, beta, U, Pold, y);
        pcg_tail<B - 1, CM>(len - k0, c, cp, odd, po, d.n - 1, v, k0, row, beta, U, Pold, y);
        return y;
    }
#endif
    static_assert(CM != 2 || PPCG_SELL_STRAIGHT, "shared offset lists are read in straight spans");
    constexpr int B = 8;
    const int64_t base = as_global(d.cptr)[chunk];
    const int len = (int)((as_global(d.cptr)[chunk + 1] - base) / kSellC);
    const PPCG_AS1 int *c = as_global(d.col + base + lane);
    const PPCG_AS1 VT *v = as_global(val + base + lane);
    T y = 0;
    for (int k0 = 0; k0 < len; k0 += B) {
        int cc[B];
        T vv[B], xx[B];
        if constexpr (C16) {
            sell_cols16<B>(d.col16, base, len, k0, lane, chunk * kSellC + lane, cc);
#pragma unroll
            for (int j = 0; j < B; ++j) {
                vv[j] = 0;
                if (k0 + j < len)
                    vv[j] = (T)stream_load(v + (size_t)(k0 + j) * kSellC);
            }
        } else {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                cc[j] = 0;
                vv[j] = 0;
                if (k0 + j < len) {
                    cc[j] = stream_load(c + (size_t)(k0 + j) * kSellC);
                    vv[j] = (T)stream_load(v + (size_t)(k0 + j) * kSellC);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < B; ++j)
            xx[j] = k0 + j < len ? U[cc[j]] + beta * Pold[cc[j]] : (T)0;
#pragma unroll
        for (int j = 0; j < B; ++j)
            if (k0 + j < len)
                y = y + vv[j] * xx[j];
    }
    return y;
}

// s = A p for one tile with p = u + beta p_old formed per gathered entry;
// returns this thread's share of (s, p).
template <typename T, typename VT>
__device__ __forceinline__ double pcg_spmv_tile(const SysDesc &d, const WorkItem wi, const VT *__restrict__ val,
                                                T beta, const PPCG_AS1 T *__restrict__ U,
                                                const PPCG_AS1 T *__restrict__ Pold, PPCG_AS1 T *__restrict__ Pnew,
                                                PPCG_AS1 T *__restrict__ S)
{
    const int n = d.n;
    double acc = 0.0;
    if (d.fmt == FMT_SELL) {
        const int lane = threadIdx.x & 63;
        const int chunk = wi.tile * kSellChunksPerTile + (threadIdx.x >> 6);
        const int i = chunk * kSellC + lane;
        if (chunk * kSellC < n) {
            // 16-bit columns measured slower for FP32 values with FP64
            // vectors (27-point case, 263 vs 242 ms), so that mix reads 32-bit ones
            const bool c16 = d.col16 && (PPCG_PCG_V32_COL16 || !(sizeof(T) == 8 && sizeof(VT) == 4));
            const T y = d.cpat ? pcg_sell_row<2>(d, val, chunk, lane, beta, U, Pold)
                        : c16  ? pcg_sell_row<1>(d, val, chunk, lane, beta, U, Pold)
                               : pcg_sell_row<0>(d, val, chunk, lane, beta, U, Pold);
            if (i < n) {
                const T pn = U[i] + beta * Pold[i];
                Pnew[i] = pn;
                S[i] = y;
                acc = acc + (double)y * (double)pn;
            }
        }
    } else {
        const int L = d.lanes;
        const int g = threadIdx.x / L, l = threadIdx.x % L;
        const int rows_per_pass = kSpmvThreads / L;
        const int passes = kTileRows / rows_per_pass;
        for (int pass = 0; pass < passes; ++pass) {
            const int i = wi.tile * kTileRows + pass * rows_per_pass + g;
            T y = 0;
            if (i < n) {
                const int e = as_global(d.rp)[i + 1];
                for (int k = as_global(d.rp)[i] + l; k < e; k += L) {
                    const int cc = stream_load(as_global(d.col + k));
                    y = y + (T)stream_load(as_global(val + k)) * (U[cc] + beta * Pold[cc]);
                }
            }
            for (int off = L >> 1; off >= 1; off >>= 1)
                y = y + __shfl_xor(y, off, 64);
            if (l == 0 && i < n) {
                const T pn = U[i] + beta * Pold[i];
                Pnew[i] = pn;
                S[i] = y;
                acc = acc + (double)y * (double)pn;
            }
        }
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(kSpmvThreads, 8) void k_pcg_spmv(const WorkItem *__restrict__ table,
                                                              const int *__restrict__ count,
                                                              const SysDesc *__restrict__ descs, int remap)
{
    __shared__ double lds[kSpmvThreads / 64];
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
    const T beta = (T)st->beta;
    const int k = st->iter;
    const PPCG_AS1 T *U = as_global((const T *)d.u);
    // beta = 0 (a start, or a restart after a breakdown): read u in place of
    // the old direction, so that whatever that buffer holds cannot leak in
    // through 0 * Inf or 0 * NaN; u + 0 u = u exactly.
    const PPCG_AS1 T *Pold = beta == (T)0 ? U : as_global((const T *)pcg_dir<T>(d, k));
    PPCG_AS1 T *Pnew = as_global(pcg_dir<T>(d, k + 1));
    PPCG_AS1 T *S = as_global((T *)d.s);
    double v[1];
    // FP32 vectors come with FP32 values (d.val); FP64 vectors use the FP32
    // copy in FP32-values mode.
    if (sizeof(T) == 4 || d.vals32)
        v[0] = pcg_spmv_tile<T, float>(d, wi, sizeof(T) == 4 ? (const float *)d.val : d.val32, beta, U, Pold,
                                       Pnew, S);
    else
        v[0] = pcg_spmv_tile<T, double>(d, wi, (const double *)d.val, beta, U, Pold, Pnew, S);
    block_sum<kSpmvThreads, 1>(v, lds);
    if (threadIdx.x == 0)
        d.part[(size_t)wi.tile * kPartStride] = v[0];  // slot 0
}

// alpha = gamma / (s, p), with breakdown when gamma <= 0, (s, p) <= 0 or a
// scalar is not finite.  One workgroup per system: the work items name
// systems (tile 0); items of other tiles exit at once, so a tile table works
// too.
__global__ __launch_bounds__(kPcgRedThreads) void k_pcg_alpha(const WorkItem *__restrict__ systab,
                                                              const int *__restrict__ count,
                                                              const SysDesc *__restrict__ descs)
{
    __shared__ double lds[kPcgRedThreads / 64];
    if ((int)blockIdx.x >= *count || systab[blockIdx.x].tile != 0)
        return;
    const SysDesc &d = descs[systab[blockIdx.x].slot];
    SysState *st = d.st;
    if (st->done)
        return;
    double dl[1];
    pcg_reduce<1>(d, 0, dl, lds);
    if (threadIdx.x == 0) {
        const double g = st->gamma, beta = st->beta;
        const double alpha = g / dl[0];
        st->delta = dl[0];
        if (!(g > 0.0) || !(dl[0] > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
            st->done = 1;
            st->status = ST_BREAKDOWN;
            return;
        }
        st->alpha = alpha;
    }
}

enum PcgUpdate { PCG_START = 0, PCG_ITER = 1, PCG_REPL = 2 };

// Stopping test at the top of Algorithm 1's loop and beta for the next
// iteration.  PCG_START follows the initialisation (beta = 0); PCG_ITER
// follows an x-update; PCG_REPL follows a reliable update: the counters stay,
// and beta = (u', r') / gamma_{i-1} with the replaced residual, the direction
// being kept.
__device__ inline void pcg_scalar_update(const SysDesc &d, SysState *st, const double (&v)[kNumPartials],
                                         int kind)
{
    if (kind == PCG_ITER) {
        st->iter += 1;
        st->i_start += 1;
        st->gamma_prev = st->gamma;
    }
    const double g = v[0], uu = v[1], rr = v[2];
    st->gamma = g;
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
    if (d.vals32 || d.prec == PREC_F32) {
        const double rn = sqrt(rr);
        if (kind != PCG_ITER) {
            st->repl_ref = rn;
        } else if (d.repl_factor > 0.0 && rn < d.repl_factor * st->repl_ref) {
            st->done = 1;
            st->status = ST_REPLACE;
            return;
        }
    }
    st->beta = kind == PCG_START || st->i_start == 0 ? 0.0 : g / st->gamma_prev;
}

template <typename T>
__global__ __launch_bounds__(kVmaThreads) void k_pcg_vma(const WorkItem *__restrict__ table,
                                                         const int *__restrict__ count,
                                                         const SysDesc *__restrict__ descs, int remap)
{
    using V2 = typename Vec2<T>::type;
    __shared__ double lds[kVmaThreads / 64 * kNumPartials];
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
    const T alpha = (T)st->alpha;
    PPCG_AS1 T *__restrict__ X = as_global((T *)d.x);
    PPCG_AS1 T *__restrict__ R = as_global((T *)d.r);
    PPCG_AS1 T *__restrict__ U = as_global((T *)d.u);
    const PPCG_AS1 T *__restrict__ P = as_global((const T *)pcg_dir<T>(d, st->iter + 1));
    const PPCG_AS1 T *__restrict__ S = as_global((const T *)d.s);
    const PPCG_AS1 T *__restrict__ DI = as_global((const T *)d.dinv);
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    auto elem = [&](T &x, T &r, T &u, T p, T sv, T di) {
        x = x + alpha * p;
        r = r - alpha * sv;
        u = di * r;
        const double rd = (double)r, ud = (double)u;
        acc[0] = acc[0] + ud * rd;
        acc[1] = acc[1] + ud * ud;
        acc[2] = acc[2] + rd * rd;
    };
    const int i = wi.tile * kTileRows + threadIdx.x * 2;
    if (i + 1 < d.n) {
        using CV2 = const PPCG_AS1 V2;
        using GV2 = PPCG_AS1 V2;
        V2 x = vload((CV2 *)(X + i)), r = vload((CV2 *)(R + i));
        const V2 p = vload((CV2 *)(P + i)), sv = vload((CV2 *)(S + i));
        // a constant diagonal: every lane reads dinv[0..1] (one cached line)
        const V2 di = vload((CV2 *)(DI + (d.dinv_const ? 0 : i)));
        V2 u;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            T xj = x[j], rj = r[j], uj;
            elem(xj, rj, uj, p[j], sv[j], di[j]);
            x[j] = xj;
            r[j] = rj;
            u[j] = uj;
        }
        vstore((GV2 *)(X + i), x);
        vstore((GV2 *)(R + i), r);
        vstore((GV2 *)(U + i), u);
    } else if (i < d.n) {
        T x = X[i], r = R[i], u;
        elem(x, r, u, P[i], S[i], DI[d.dinv_const ? 0 : i]);
        X[i] = x;
        R[i] = r;
        U[i] = u;
    }
    block_sum<kVmaThreads, kNumPartials>(acc, lds);
    if (threadIdx.x == 0) {
        double *out = d.part + ((size_t)d.ntiles + wi.tile) * kPartStride;  // slot 1
        for (int k = 0; k < kNumPartials; ++k)
            out[k] = acc[k];
    }
}

// After r = b - A x and u = M^-1 r were (re)computed (MODE_INIT1 at a start,
// MODE_REPL1 at a reliable update): partial sums of (u, r), (u, u), (r, r)
// and (b, b) per tile, in the layout k_pcg_update reduces.
template <typename T>
__global__ __launch_bounds__(kVmaThreads) void k_pcg_dots(const WorkItem *__restrict__ table,
                                                          const int *__restrict__ count,
                                                          const SysDesc *__restrict__ descs)
{
    __shared__ double lds[kVmaThreads / 64 * kNumPartials];
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    const T *__restrict__ R = (const T *)d.r;
    const T *__restrict__ U = (const T *)d.u;
    const T *__restrict__ Bv = (const T *)d.b;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 2; ++k) {
        const int i = wi.tile * kTileRows + threadIdx.x * 2 + k;
        if (i < d.n) {
            const double ui = (double)U[i], ri = (double)R[i], bi = (double)Bv[i];
            acc[0] = acc[0] + ui * ri;
            acc[1] = acc[1] + ui * ui;
            acc[2] = acc[2] + ri * ri;
            acc[3] = acc[3] + bi * bi;
        }
    }
    block_sum<kVmaThreads, kNumPartials>(acc, lds);
    if (threadIdx.x == 0) {
        double *out = d.part + ((size_t)d.ntiles + wi.tile) * kPartStride;  // slot 1
        for (int k = 0; k < kNumPartials; ++k)
            out[k] = acc[k];
    }
}

// Reduce the update's partial sums and run the scalar update of the given
// kind.  One workgroup per system.  After k_pcg_vma (PCG_ITER) only systems
// still iterating take part; after k_pcg_dots (PCG_START, PCG_REPL) the
// system's state is set up again, (b, b) included.
template <int KIND>
__global__ __launch_bounds__(kPcgRedThreads) void k_pcg_update(const WorkItem *__restrict__ systab,
                                                               const int *__restrict__ count,
                                                               const SysDesc *__restrict__ descs)
{
    __shared__ double lds[kPcgRedThreads / 64 * kNumPartials];
    if ((int)blockIdx.x >= *count || systab[blockIdx.x].tile != 0)
        return;
    const SysDesc &d = descs[systab[blockIdx.x].slot];
    SysState *st = d.st;
    if (KIND == PCG_ITER && st->done)
        return;
    double v[kNumPartials];
    pcg_reduce<kNumPartials>(d, 1, v, lds);
    if (threadIdx.x == 0) {
        if (KIND != PCG_ITER) {
            st->bnorm2 = v[3];
            st->phase = 0;
        }
        // A reliable update after a breakdown restarts the direction (beta = 0)
        // from the replaced residual: the kept direction is not usable.
        if (KIND == PCG_REPL && st->status == ST_BREAKDOWN)
            st->i_start = 0;
        pcg_scalar_update(d, st, v, KIND);
    }
}

// FP32 mixed precision with classic PCG, end of an inner stretch:
// x64 += c x32 with c = ||r64|| at the last k_pcg_mix_start, and c is kept
// (in the FP64 slot's repl_ref) for the rescaling at the next start.  Work
// items name FP64 slots; SysDesc::pair is the FP32 slot.
__global__ void k_pcg_mix_correct(const WorkItem *__restrict__ table, const int *__restrict__ count,
                                  const SysDesc *__restrict__ d64, const SysDesc *__restrict__ d32)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &a = d64[wi.slot];
    const SysDesc &f = d32[a.pair];
    const double c = sqrt(a.st->tnorm2);
    double *__restrict__ x = (double *)a.x;
    const float *__restrict__ x32 = (const float *)f.x;
    for (int k = threadIdx.x; k < kTileRows; k += blockDim.x) {
        const int i = wi.tile * kTileRows + k;
        if (i < a.n)
            x[i] = x[i] + c * (double)x32[i];
    }
    if (wi.tile == 0 && threadIdx.x == 0)
        a.st->repl_ref = c;  // no workgroup of this launch reads repl_ref
}

// Start (or continue) the FP32 sequence on b32 = r64 / ||r64||, x32 = 0.
// When the FP32 slot holds a live direction (i_start > 0), the system was
// scaled by 1 / c_old: in the new units y' = (c_old / c_new) y, so the current
// direction is multiplied by c_old / c_new and gamma_{i-1} by its square;
// beta = gamma' / gamma_{i-1} of the following reliable update is then the
// one of the unscaled iteration.
__global__ void k_pcg_mix_start(const WorkItem *__restrict__ table, const int *__restrict__ count,
                                const SysDesc *__restrict__ d64, const SysDesc *__restrict__ d32)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &a = d64[wi.slot];
    const SysDesc &f = d32[a.pair];
    const double cn = sqrt(a.st->tnorm2);
    const double inv = 1.0 / cn;
    const bool live = f.st->i_start > 0;
    const float scale = live ? (float)(a.st->repl_ref / cn) : 1.0f;
    float *__restrict__ P = pcg_dir<float>(f, f.st->iter);
    const double *__restrict__ r = (const double *)a.r;
    float *__restrict__ b32 = (float *)f.b;
    float *__restrict__ x32 = (float *)f.x;
    for (int k = threadIdx.x; k < kTileRows; k += blockDim.x) {
        const int i = wi.tile * kTileRows + k;
        if (i < a.n) {
            b32[i] = (float)(r[i] * inv);
            x32[i] = 0.0f;
            if (live)
                P[i] = P[i] * scale;
        }
    }
    if (live && wi.tile == 0 && threadIdx.x == 0) {
        const double c = a.st->repl_ref / cn;
        f.st->gamma_prev = f.st->gamma_prev * c * c;  // no workgroup of this launch reads gamma_prev
    }
}

}  // namespace ppcg
