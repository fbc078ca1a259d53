// ppcg_pcg.hpp -- classic PCG (Algorithm 1 of Tiwari & Vadhiyar, Section
// III-A) on the device, for comparison with the pipelined method, and as the
// iteration of the FP32-values mode when selected.
//
// One iteration is two launches over the same (system, tile) work table:
//
//   k_pcg_spmv<PAR>  p = u + beta p (formed on the fly for every gathered
//                    entry, written for the workgroup's own rows into the
//                    other buffer of a double-buffered pair), s = A p, and
//                    the partial sums of (s, p); the last workgroup to finish
//                    (arrival ticket) reduces them and computes alpha.
//   k_pcg_vma<PAR>   x += alpha p, r -= alpha s, u = M^-1 r and the partial
//                    sums of (u, r), (u, u), (r, r); the last workgroup
//                    reduces them, runs the stopping test and computes beta.
//
// Unlike Algorithm 2, each iteration has two reductions that the next launch
// depends on, so they are done by the last-arriving workgroup.  PAR selects
// which of p / z holds the previous direction; iterations alternate PAR.
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

// Last-workgroup reduction: every workgroup publishes its record, then
// increments the system's ticket; the one that brings it to ntiles reduces
// all records in tile order.  Returns true (in every thread) for that one.
__device__ __forceinline__ bool arrive_last(const SysDesc &d, SysState *st, int *flag)
{
    __syncthreads();  // this workgroup's partial record is written (thread 0)
    if (threadIdx.x == 0) {
        __threadfence();  // publish the record before arriving
        const int t = atomicAdd(&st->ticket, 1);
        *flag = (t == d.ntiles - 1);
    }
    __syncthreads();
    const bool last = *flag != 0;
    if (last)
        __threadfence();  // acquire: see every other workgroup's record
    return last;
}

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

template <int PAR>
__global__ __launch_bounds__(kSpmvThreads, 8) void k_pcg_spmv(const WorkItem *__restrict__ table,
                                                              const int *__restrict__ count,
                                                              const SysDesc *__restrict__ descs, int remap)
{
    __shared__ double lds[kSpmvThreads / 64];
    __shared__ int flag;
    const int pos = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    SysState *st = d.st;
    if (st->done)
        return;
    const double beta = st->beta;
    const double *U = (const double *)d.u;
    const double *Pold = (const double *)(PAR ? d.z : d.p);
    double *Pnew = (double *)(PAR ? d.p : d.z);
    double *S = (double *)d.s;
    double v[1];
    if (d.vals32)
        v[0] = pcg_spmv_tile<float>(d, wi, d.val32, beta, U, Pold, Pnew, S);
    else
        v[0] = pcg_spmv_tile<double>(d, wi, (const double *)d.val, beta, U, Pold, Pnew, S);
    block_sum<kSpmvThreads, 1>(v, lds);
    if (threadIdx.x == 0)
        d.part[(size_t)wi.tile * kPartStride] = v[0];  // slot 0
    if (!arrive_last(d, st, &flag))
        return;
    double dl[1];
    reduce_partials<kSpmvThreads, 1>(d, 0, dl, lds);
    if (threadIdx.x == 0) {
        st->ticket = 0;
        const double g = st->gamma;
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
// iteration (thread 0 of the last workgroup).  PCG_START follows the
// initialisation (beta = 0); PCG_ITER follows an x-update; PCG_REPL follows a
// reliable update: the counters stay, and beta = (u', r') / gamma_{i-1} with
// the replaced residual, the direction being kept.
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

template <int PAR>
__global__ __launch_bounds__(kVmaThreads) void k_pcg_vma(const WorkItem *__restrict__ table,
                                                         const int *__restrict__ count,
                                                         const SysDesc *__restrict__ descs, int remap)
{
    __shared__ double lds[kVmaThreads / 64 * kNumPartials];
    __shared__ int flag;
    const int pos = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    SysState *st = d.st;
    if (st->done)
        return;
    const double alpha = st->alpha;
    double *__restrict__ X = (double *)d.x;
    double *__restrict__ R = (double *)d.r;
    double *__restrict__ U = (double *)d.u;
    const double *__restrict__ P = (const double *)(PAR ? d.p : d.z);
    const double *__restrict__ S = (const double *)d.s;
    const double *__restrict__ DI = (const double *)d.dinv;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 2; ++k) {
        const int i = wi.tile * kTileRows + threadIdx.x * 2 + k;
        if (i < d.n) {
            const double x = X[i] + alpha * P[i];
            const double r = R[i] - alpha * S[i];
            const double u = DI[i] * r;
            X[i] = x;
            R[i] = r;
            U[i] = u;
            acc[0] = acc[0] + u * r;
            acc[1] = acc[1] + u * u;
            acc[2] = acc[2] + r * r;
        }
    }
    block_sum<kVmaThreads, kNumPartials>(acc, lds);
    if (threadIdx.x == 0) {
        double *out = d.part + ((size_t)d.ntiles + wi.tile) * kPartStride;  // slot 1
        for (int k = 0; k < kNumPartials; ++k)
            out[k] = acc[k];
    }
    if (!arrive_last(d, st, &flag))
        return;
    double v[kNumPartials];
    reduce_partials<kVmaThreads>(d, 1, v, lds);
    if (threadIdx.x == 0) {
        st->ticket = 0;
        pcg_scalar_update(d, st, v, PCG_ITER);
    }
}

// After r = b - A x and u = M^-1 r were (re)computed (MODE_INIT1 at a start,
// MODE_REPL1 at a reliable update): (u, r), (u, u), (r, r), (b, b) and the
// scalar update of the given kind (PCG_START or PCG_REPL).
template <int KIND>
__global__ __launch_bounds__(kVmaThreads) void k_pcg_restart(const WorkItem *__restrict__ table,
                                                             const int *__restrict__ count,
                                                             const SysDesc *__restrict__ descs)
{
    __shared__ double lds[kVmaThreads / 64 * kNumPartials];
    __shared__ int flag;
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    SysState *st = d.st;
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
    if (!arrive_last(d, st, &flag))
        return;
    double v[kNumPartials];
    reduce_partials<kVmaThreads>(d, 1, v, lds);
    if (threadIdx.x == 0) {
        st->ticket = 0;
        st->bnorm2 = v[3];
        st->phase = 0;
        // A reliable update after a breakdown restarts the direction (beta = 0)
        // from the replaced residual: the kept direction is not usable.
        if (KIND == PCG_REPL && st->status == ST_BREAKDOWN)
            st->i_start = 0;
        pcg_scalar_update(d, st, v, KIND);
    }
}

}  // namespace ppcg
