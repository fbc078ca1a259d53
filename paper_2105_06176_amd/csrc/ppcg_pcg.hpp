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

// Fixed-order reduction of NV partials over a system's tiles for the
// one-workgroup reduction kernels: thread t takes the tiles t, t + NT, ...
// in index order, with the loads of kPcgRedBatch tiles issued before their
// sums (one memory latency per batch), then the workgroup tree.
constexpr int kPcgRedBatch = 4;

template <int NV>
__device__ __forceinline__ void pcg_reduce(const SysDesc &d, int slot, double (&out)[NV], double *lds)
{
    const double *P = d.part + (size_t)slot * d.ntiles * kPartStride;
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

// Direction buffers: the current direction after k x-updates is in pbuf(k).
__device__ __forceinline__ double *pcg_dir(const SysDesc &d, int k) { return (double *)((k & 1) ? d.z : d.p); }

// s = A p for one tile with p = u + beta p_old formed per gathered entry;
// returns this thread's share of (s, p).
template <typename VT>
__device__ __forceinline__ double pcg_spmv_tile(const SysDesc &d, const WorkItem wi, const VT *__restrict__ val,
                                                double beta, const double *__restrict__ U,
                                                const double *__restrict__ Pold, double *__restrict__ Pnew,
                                                double *__restrict__ S)
{
    const int n = d.n;
    double acc = 0.0;
    if (d.fmt == FMT_SELL) {
        const int lane = threadIdx.x & 63;
        const int chunk = wi.tile * kSellChunksPerTile + (threadIdx.x >> 6);
        const int i = chunk * kSellC + lane;
        if (chunk * kSellC < n) {
            constexpr int B = 8;
            const int64_t base = d.cptr[chunk];
            const int len = (int)((d.cptr[chunk + 1] - base) / kSellC);
            const int *c = d.col + base + lane;
            const VT *v = val + base + lane;
            double y = 0.0;
            for (int k0 = 0; k0 < len; k0 += B) {
                int cc[B];
                double vv[B], xx[B];
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    cc[j] = 0;
                    vv[j] = 0.0;
                    if (k0 + j < len) {
                        cc[j] = stream_load(c + (size_t)(k0 + j) * kSellC);
                        vv[j] = (double)stream_load(v + (size_t)(k0 + j) * kSellC);
                    }
                }
#pragma unroll
                for (int j = 0; j < B; ++j)
                    xx[j] = k0 + j < len ? U[cc[j]] + beta * Pold[cc[j]] : 0.0;
#pragma unroll
                for (int j = 0; j < B; ++j)
                    if (k0 + j < len)
                        y = y + vv[j] * xx[j];
            }
            if (i < n) {
                const double pn = U[i] + beta * Pold[i];
                Pnew[i] = pn;
                S[i] = y;
                acc = acc + y * pn;
            }
        }
    } else {
        const int L = d.lanes;
        const int g = threadIdx.x / L, l = threadIdx.x % L;
        const int rows_per_pass = kSpmvThreads / L;
        const int passes = kTileRows / rows_per_pass;
        for (int pass = 0; pass < passes; ++pass) {
            const int i = wi.tile * kTileRows + pass * rows_per_pass + g;
            double y = 0.0;
            if (i < n) {
                const int e = d.rp[i + 1];
                for (int k = d.rp[i] + l; k < e; k += L) {
                    const int cc = stream_load(d.col + k);
                    y = y + (double)stream_load(val + k) * (U[cc] + beta * Pold[cc]);
                }
            }
            for (int off = L >> 1; off >= 1; off >>= 1)
                y = y + __shfl_xor(y, off, 64);
            if (l == 0 && i < n) {
                const double pn = U[i] + beta * Pold[i];
                Pnew[i] = pn;
                S[i] = y;
                acc = acc + y * pn;
            }
        }
    }
    return acc;
}

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
    const double beta = st->beta;
    const int k = st->iter;
    const double *U = (const double *)d.u;
    const double *Pold = pcg_dir(d, k);
    double *Pnew = pcg_dir(d, k + 1);
    double *S = (double *)d.s;
    double v[1];
    if (d.vals32)
        v[0] = pcg_spmv_tile<float>(d, wi, d.val32, beta, U, Pold, Pnew, S);
    else
        v[0] = pcg_spmv_tile<double>(d, wi, (const double *)d.val, beta, U, Pold, Pnew, S);
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
    st->gen += 1;
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
    if (d.vals32) {
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

__global__ __launch_bounds__(kVmaThreads) void k_pcg_vma(const WorkItem *__restrict__ table,
                                                         const int *__restrict__ count,
                                                         const SysDesc *__restrict__ descs, int remap)
{
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
    const double alpha = st->alpha;
    double *__restrict__ X = (double *)d.x;
    double *__restrict__ R = (double *)d.r;
    double *__restrict__ U = (double *)d.u;
    const double *__restrict__ P = pcg_dir(d, st->iter + 1);
    const double *__restrict__ S = (const double *)d.s;
    const double *__restrict__ DI = (const double *)d.dinv;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    auto elem = [&](double &x, double &r, double &u, double p, double sv, double di) {
        x = x + alpha * p;
        r = r - alpha * sv;
        u = di * r;
        acc[0] = acc[0] + u * r;
        acc[1] = acc[1] + u * u;
        acc[2] = acc[2] + r * r;
    };
    const int i = wi.tile * kTileRows + threadIdx.x * 2;
    if (i + 1 < d.n) {
        dvec2 x = vload((const dvec2 *)(X + i)), r = vload((const dvec2 *)(R + i));
        const dvec2 p = vload((const dvec2 *)(P + i)), sv = vload((const dvec2 *)(S + i));
        // a constant diagonal: every lane reads dinv[0..1] (one cached line)
        const dvec2 di = vload((const dvec2 *)(DI + (d.dinv_const ? 0 : i)));
        dvec2 u;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double xj = x[j], rj = r[j], uj;
            elem(xj, rj, uj, p[j], sv[j], di[j]);
            x[j] = xj;
            r[j] = rj;
            u[j] = uj;
        }
        vstore((dvec2 *)(X + i), x);
        vstore((dvec2 *)(R + i), r);
        vstore((dvec2 *)(U + i), u);
    } else if (i < d.n) {
        double x = X[i], r = R[i], u;
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
    const double *__restrict__ R = (const double *)d.r;
    const double *__restrict__ U = (const double *)d.u;
    const double *__restrict__ Bv = (const double *)d.b;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 2; ++k) {
        const int i = wi.tile * kTileRows + threadIdx.x * 2 + k;
        if (i < d.n) {
            acc[0] = acc[0] + U[i] * R[i];
            acc[1] = acc[1] + U[i] * U[i];
            acc[2] = acc[2] + R[i] * R[i];
            acc[3] = acc[3] + Bv[i] * Bv[i];
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

}  // namespace ppcg
