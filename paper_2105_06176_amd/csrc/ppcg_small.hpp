// ppcg_small.hpp -- one-workgroup PIPECG iteration kernel for small systems
// (Algorithm 2 of Tiwari & Vadhiyar, Section III-B, the same arithmetic as
// the fused update + SpMV pair of ppcg_kernels.hpp).
#pragma once

#include "ppcg_kernels.hpp"

namespace ppcg {

// ---------------------------------------------------------------------------
// Small systems: one workgroup of kSmallThreads runs up to `iters` whole
// PIPECG iterations of one system per launch (work item = system).  Thread t
// owns the rows t, t + kSmallThreads, ... (at most kSmallRowsPerThread) and
// keeps their z, q, s, p, r, u, w and n in registers for the whole launch;
// m, the only vector other rows read (the SpMV gathers), and x live in LDS,
// the scalar state record in LDS, the chunk extents in scalar registers.  An iteration touches global memory only for the matrix
// and an inverse diagonal that is not constant (L2-resident at these sizes):
// fused update, fixed-order workgroup reduction and scalar update (thread 0),
// workgroup barrier, SpMV from LDS, barrier.  Vectors and the state are
// loaded at the start and stored at the end of the launch, so the state in
// HBM is complete between launches.  SELL
// format only; rows of a wavefront form one SELL chunk, so chunk lengths are
// uniform across each wavefront.
//
// With the one-byte value table (the matrix has at most 256 distinct values)
// and at most kSmallLdsEntries stored entries, the matrix itself is staged
// in LDS at the start of the launch, each entry as a 16-bit column offset
// from its row and its value index: the SpMV of an iteration then reads
// nothing from global memory, and its steps over a row's entries wait on
// LDS instead of L2 round trips.  Same values and order, so the same sums.
constexpr int kSmallThreads = 512;
constexpr int kSmallRowsPerThread = 8;
constexpr int kSmallMaxRows = kSmallThreads * kSmallRowsPerThread;
constexpr int kSmallLdsEntries = 24576;
static_assert(kSmallMaxRows <= 32768, "column offsets from the row fit 16 bits");
static_assert(PPCG_SMALL_MAX_ROWS <= kSmallMaxRows, "small systems must fit the register-resident kernel");

__global__ __launch_bounds__(kSmallThreads) void k_small_iter(const WorkItem *__restrict__ table,
                                                              const int *__restrict__ count,
                                                              const SysDesc *__restrict__ descs, int iters)
{
    constexpr int R = kSmallRowsPerThread;
    __shared__ double lds[kSmallThreads / 64 * kNumPartials];
    __shared__ double lm[kSmallMaxRows];  // m
    __shared__ double lx[kSmallMaxRows];  // x, written back at the end of the launch
    __shared__ double scal[2];            // alpha, beta of the next update
    __shared__ SysState loc;              // the state record, written back at the end of the launch
    __shared__ int stop;
    __shared__ short lco[kSmallLdsEntries];           // staged matrix: column - row
    __shared__ unsigned char lvi[kSmallLdsEntries];   // and value index
    __shared__ double ltab[kMaxValueTable];           // the value table
    if ((int)blockIdx.x >= *count)
        return;
    const WorkItem wi = table[blockIdx.x];
    const SysDesc &d = descs[wi.slot];
    SysState *st = d.st;
    const int n = d.n;
    double *__restrict__ X = (double *)d.x;
    double *__restrict__ Rv = (double *)d.r;
    double *__restrict__ U = (double *)d.u;
    double *__restrict__ W = (double *)d.w;
    double *__restrict__ M = (double *)d.m;
    double *__restrict__ NVv = (double *)d.nv;
    double *__restrict__ Z = (double *)d.z;
    double *__restrict__ S = (double *)d.s;
    double *__restrict__ P = (double *)d.p;
    const double *__restrict__ DI = (const double *)d.dinv;
    const double *__restrict__ val = (const double *)d.val;
    const int *__restrict__ col = d.col;
    const int64_t *__restrict__ cptr = d.cptr;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // u and q are scalings of r and s by the inverse diagonal (see vma_elem):
    // u is formed from r, q never
    double z[R], s[R], p[R], r[R], u[R], w[R], nv[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = threadIdx.x + j * kSmallThreads;
        const bool ok = i < n;
        z[j] = ok ? Z[i] : 0.0;
        s[j] = ok ? S[i] : 0.0;
        p[j] = ok ? P[i] : 0.0;
        r[j] = ok ? Rv[i] : 0.0;
        u[j] = ok ? U[i] : 0.0;  // written back unchanged if no iteration runs
        w[j] = ok ? W[i] : 0.0;
        nv[j] = ok ? NVv[i] : 0.0;
        if (ok) {
            lm[i] = M[i];
            lx[i] = X[i];
        }
    }
    // The state record lives in LDS for the launch (written back at its end),
    // the chunk extents in scalar registers.
    if (threadIdx.x == 0) {
        loc = *st;
        stop = loc.done;
        scal[0] = loc.alpha;
        scal[1] = loc.beta;
    }
    int base[R], len[R], maxlen = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int c = wave + j * (kSmallThreads / 64);
        base[j] = 0;
        len[j] = 0;
        if (c * kSellC < n) {  // c is the same in every lane: scalar registers
            base[j] = __builtin_amdgcn_readfirstlane((int)cptr[c]);
            len[j] = __builtin_amdgcn_readfirstlane((int)((cptr[c + 1] - cptr[c]) / kSellC));
        }
        maxlen = len[j] > maxlen ? len[j] : maxlen;
    }
    const bool dconst = d.dinv_const != 0;
    const double d0 = DI[0];
    // staged matrix (uniform over the workgroup)
    const bool staged = d.vidx != nullptr && cptr[(n + kSellC - 1) / kSellC] <= kSmallLdsEntries;
    if (staged) {
        for (int t = threadIdx.x; t < d.nvtab; t += kSmallThreads)
            ltab[t] = d.vtab[t];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int row = threadIdx.x + j * kSmallThreads;
            for (int k = 0; k < len[j]; ++k) {
                const int o = base[j] + lane + k * kSellC;
                lco[o] = (short)(col[o] - row);
                lvi[o] = d.vidx[o];
            }
        }
    }
    __syncthreads();
    for (int it = 0; it < iters && !stop; ++it) {
        const double sa = scal[0], sb = scal[1];
        double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
        // the inverse diagonal: one value, or loaded first (one memory latency)
        double dg[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = threadIdx.x + j * kSmallThreads;
            dg[j] = d0;
            if (!dconst && i < n)
                dg[j] = DI[i];
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = threadIdx.x + j * kSmallThreads;
            if (i < n) {
                double mo;
                vma_elem<double, kNumPartials>(sa, sb, nv[j], z[j], w[j], s[j], p[j], r[j], dg[j], u[j], mo, acc);
                lx[i] = lx[i] + sa * p[j];  // this kernel updates x every iteration
                lm[i] = mo;  // only this thread touches lm[i] and lx[i] until the barrier below
            }
        }
        block_sum<kSmallThreads, kNumPartials>(acc, lds);
        if (threadIdx.x == 0) {
            scalar_update<kNumPartials>(d, &loc, acc);
            stop = loc.done;
            scal[0] = loc.alpha;
            scal[1] = loc.beta;
        }
        __syncthreads();  // m complete in LDS; the new scalars visible
        // SpMV from LDS: the wavefront's chunk for row slot j is wave + j *
        // (waves per workgroup); entry k of all its chunks is fetched together.
        // (stored entries of a system with at most kSmallMaxRows rows fit 32 bits)
#pragma unroll
        for (int j = 0; j < R; ++j)
            nv[j] = 0.0;
        if (staged) {
            for (int k = 0; k < maxlen; ++k) {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if (k < len[j]) {
                        const int o = base[j] + lane + k * kSellC;
                        nv[j] = nv[j] + ltab[lvi[o]] * lm[threadIdx.x + j * kSmallThreads + lco[o]];
                    }
                }
            }
        }
        for (int k = 0; k < (staged ? 0 : maxlen); ++k) {
            // entry k of every row slot: loads first, then the LDS gathers
            int cv[R];
            double vv[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                cv[j] = 0;
                vv[j] = 0.0;
                if (k < len[j]) {
                    const size_t o = (size_t)base[j] + lane + (size_t)k * kSellC;
                    cv[j] = col[o];
                    vv[j] = val[o];
                }
            }
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (k < len[j])
                    nv[j] = nv[j] + vv[j] * lm[cv[j]];
        }
        __syncthreads();  // every gather of m done before the next update rewrites it
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = threadIdx.x + j * kSmallThreads;
        if (i < n) {
            Z[i] = z[j];
            S[i] = s[j];
            P[i] = p[j];
            Rv[i] = r[j];
            U[i] = u[j];
            W[i] = w[j];
            NVv[i] = nv[j];
            M[i] = lm[i];
            X[i] = lx[i];
        }
    }
    if (threadIdx.x == 0)
        *st = loc;
}

}  // namespace ppcg
