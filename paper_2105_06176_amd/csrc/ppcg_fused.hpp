// ppcg_fused.hpp -- the PIPECG iteration of Algorithm 2 (Tiwari & Vadhiyar,
// Section III-B) as ONE launch per iteration.
//
// The two-launch form (ppcg_kernels.hpp) writes n = A m in the SpMV launch
// and reads it back in the next fused update.  Here each workgroup owns a
// tile of frows rows (512 to 8,192, fused_tile_rows: 1 to 16 rows per
// thread, chosen by the tile count and the compute units) and, in one
// launch:
//
//   0. computes its first row of n = A m_i (which needs none of this
//      launch's scalars), so that the latency of that SpMV overlaps step 1;
//   1. reduces, in one fixed order, the per-tile partial sums of (r,u),
//      (w,u), (u,u), (r,r) that the previous launch wrote, and runs the scalar
//      recurrences (the stopping test, beta, alpha, breakdown) itself: every
//      workgroup reads the same partials in the same order and so obtains
//      bit-identical scalars, with no grid-wide synchronisation;
//   2. for each of its rows (SELL-64, one lane per row, up to
//      kFusedRowsPerThread rows per thread) computes n = A m_i into a
//      register and applies the fused vector updates of Section V-B with
//      it.  With a constant diagonal m_i = M^-1 w_i is not stored: the SpMV
//      gathers w_i and forms each m_i[col] = dinv[0] * w_i[col] itself, the
//      same rounded product the update would have stored;
//   3. writes its own partial sums.
//
// The kernel boundary is the only synchronisation.  Everything another
// workgroup of the same launch may still read is double buffered by the
// launch's parity `par`: what the SpMV gathers of every tile read (w, or m
// for a diagonal that is not constant), the partial sums and the scalar
// state record.  Launch j of a captured chunk has par = j & 1 and chunks
// have an even number of launches, so a running system always starts a
// chunk with that vector in buffer 0 (the handle's own w or m vector)
// and its latest partials and state in slot 0; k_fused_begin, the first
// node of every chunk, copies the canonical state record into slot 0 and,
// right after an initialisation, folds the initialisation's 512-row
// partials into the fused tiles' partials.
//
// Per iteration this saves the n round trip (16 bytes per row), with a
// constant diagonal the m write (8 bytes per row), and one launch.  The cost
// is the partial-sum reduction every workgroup repeats: 32 bytes per tile,
// read from the L2 (512 tiles of 4,096 rows at 2^21 rows: 16 KB per
// workgroup).
//
// The arithmetic of one row is that of the two-launch form (same SpMV order,
// same products, same update formulas, x-updates paired in the same way);
// only the association of the dot products differs (over the fused tiles),
// so results are deterministic, identical alone and batched, but not bitwise
// equal to the two-launch form.
#pragma once

#include "ppcg_kernels.hpp"

namespace ppcg {

// Waves per SIMD the kernel is compiled for: 4 lets it keep its 76 VGPRs
// (6 waves per SIMD in practice); forcing 8 spills and was 14 % slower.
#ifndef PPCG_FUSED_WAVES
#define PPCG_FUSED_WAVES 4
#endif
// 1: a thread's first row gets its SpMV before the reduction of the previous
// partials and the scalar update (it does not depend on this launch's
// scalars), so its latency overlaps that chain.
#ifndef PPCG_FUSED_ROW0_EARLY
#define PPCG_FUSED_ROW0_EARLY 1
#endif
// XCD-aware tile order (each XCD a contiguous range of tiles): 1.7 % faster
// on the 128^3 7-point system.
#ifndef PPCG_FUSED_REMAP
#define PPCG_FUSED_REMAP 1
#endif

// The 64-bit value that lane j holds, in scalar registers (j uniform).
__device__ __forceinline__ int64_t lane_i64(int64_t v, int j)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(uint64_t)v, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((uint64_t)v >> 32), j);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

struct FusedScalars {
    double alpha, beta, alpha_x;
    int go, x_pending, x_finish;
};

// SpMV of one SELL chunk row with the handle's storage variant.  SC = 1: on
// m formed from w on the fly, n_row = sum over the row's entries of
// a * (d0 * w[col]), each d0 * w[col] the same rounded product the update
// forms for m (a constant diagonal, d0 = dinv[0]); SC = 0: on m as stored.
template <int SC>
__device__ __forceinline__ double fused_row_sc(const SysDesc &d, const double *win, int chunk, int lane,
                                               const double *tab, const double *dg, double d0, int64_t eb, int el,
                                               int ep)
{
    const double *xin[1] = {win};
    double y[1];
    const double *val = (const double *)d.val;
    if (d.cpat) {
        if (tab)
            sell_row_shared<double, double, 1, true, SC>(d.cptr, d.cpat, d.pats, val, xin, chunk, lane, d.n, y,
                                                         d.vidx, tab, dg, d0, eb, el, ep);
        else
            sell_row_shared<double, double, 1, false, SC>(d.cptr, d.cpat, d.pats, val, xin, chunk, lane, d.n, y,
                                                          nullptr, nullptr, dg, d0, eb, el, ep);
        return y[0];
    }
    if (tab) {
        if (d.col16)
#if PPCG_SELL_PIPE
            sell_row16_pipe<double, double, 1, true, SC>(d.cptr, d.col16, val, xin, chunk, lane, y, d.vidx, tab, dg,
                                                         d0, eb, el);
#else
            sell_row16<double, double, 1, true, SC>(d.cptr, d.col16, val, xin, chunk, lane, y, d.vidx, tab, dg, d0,
                                                    eb, el);
#endif
        else
            sell_row<double, double, 1, true, SC>(d.cptr, d.col, val, xin, chunk, lane, y, d.vidx, tab, dg, d0, eb,
                                                  el);
    } else {
        if (d.col16)
#if PPCG_SELL_PIPE
            sell_row16_pipe<double, double, 1, false, SC>(d.cptr, d.col16, val, xin, chunk, lane, y, nullptr, nullptr,
                                                          dg, d0, eb, el);
#else
            sell_row16<double, double, 1, false, SC>(d.cptr, d.col16, val, xin, chunk, lane, y, nullptr, nullptr, dg,
                                                     d0, eb, el);
#endif
        else
            sell_row<double, double, 1, false, SC>(d.cptr, d.col, val, xin, chunk, lane, y, nullptr, nullptr, dg, d0,
                                                   eb, el);
    }
    return y[0];
}

// Systems whose diagonal is constant gather w and scale it (m is never
// stored); others gather the stored m.  (Gathering dinv next to w for a
// general diagonal needs 14 more VGPRs in this kernel: 88 against 74, one
// wavefront per SIMD fewer for every system.)  eb, el: the chunk's first
// stored slot and padded length; ep: the start of its shared offset list.
__device__ __forceinline__ double fused_row(const SysDesc &d, const double *gin, int chunk, int lane,
                                            const double *tab, int64_t eb, int el, int ep)
{
    if (d.dinv_const)
        return fused_row_sc<1>(d, gin, chunk, lane, tab, nullptr, ((const double *)d.dinv)[0], eb, el, ep);
    return fused_row_sc<0>(d, gin, chunk, lane, tab, nullptr, 0.0, eb, el, ep);
}

__global__ __launch_bounds__(kFusedThreads, PPCG_FUSED_WAVES) void k_fused(const WorkItem *__restrict__ table,
                                                                           const int *__restrict__ count,
                                                                           const SysDesc *__restrict__ descs,
                                                                           int remap, int par)
{
    __shared__ double lds[kFusedThreads / 64 * kNumPartials];
    __shared__ double vtab[kMaxValueTable];
    __shared__ FusedScalars sc;
    const int live = *count;
    if ((int)blockIdx.x >= live)
        return;
    const int pos = remap ? xcd_remap(blockIdx.x, live) : (int)blockIdx.x;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    const int R = d.frows / kFusedThreads;  // rows per thread, 1 .. kFusedRowsPerThread
    const SysState *rin = d.frec + par;
    const int n = d.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row0 = wi.tile * d.frows;
    // Loads that need only the descriptor are issued before the stop check,
    // so that their latencies overlap instead of following one another:
    // the extents of this wavefront's chunks (row k of a thread lies in chunk
    // c0 + k * kFusedThreads / 64: lane j < 2R holds cptr[c0 + (j >> 1) * 8 +
    // (j & 1)]) and, with shared offset lists, the lists' starts (lane
    // 32 + k < 32 + R holds cpat[c0 + k * 8]), this thread's first two
    // partial-sum records, and its entry of the value table.
    static_assert(2 * kFusedRowsPerThread <= 32, "extents in lanes 0 .. 31, list starts in lanes 32 .. 63");
    int64_t ext = 0;
    int pst = 0;
    {
        const int c0 = row0 / kSellC + wave;
        const int nch = (n + kSellC - 1) / kSellC;
        const int j = lane >> 1, e = lane & 1;
        const int c = c0 + j * (kFusedThreads / kSellC) + e;
        if (j < R && c <= nch)
            ext = as_global(d.cptr)[c];
        const int kp = lane - 32;
        const int cp = c0 + kp * (kFusedThreads / kSellC);
        if (d.cpat && kp >= 0 && kp < R && cp < nch)
            pst = as_global(d.cpat)[cp];
    }
    const int nft = d.nftiles;
    const PPCG_AS1 dvec2 *PR = (const PPCG_AS1 dvec2 *)as_global(d.fpart + (size_t)par * nft * 4);
    dvec2 pa0 = {0.0, 0.0}, pb0 = {0.0, 0.0}, pa1 = {0.0, 0.0}, pb1 = {0.0, 0.0};
    const bool has0 = tid < nft, has1 = tid + kFusedThreads < nft;
    if (has0) {
        pa0 = PR[2 * tid];
        pb0 = PR[2 * tid + 1];
    }
    if (has1) {
        pa1 = PR[2 * (tid + kFusedThreads)];
        pb1 = PR[2 * (tid + kFusedThreads) + 1];
    }
    static_assert(kMaxValueTable <= kFusedThreads, "one value-table entry per thread");
    const bool vt = d.vidx != nullptr;
    double tv = 0.0;
    if (vt && tid < d.nvtab)
        tv = d.vtab[tid];
    __asm__ volatile("" ::: "memory");  // the loads above stay above the check
    if (rin->done) {
        // The launch that stopped the system published its record in this
        // launch's slot only.  Copy it into the other slot, so that the
        // launch after this one also sees it: otherwise that launch would
        // redo the stopping step from the older record (and apply the final
        // x-update a second time).  Nothing in this launch reads the other slot.
        if (wi.tile == 0 && threadIdx.x == 0)
            d.frec[par ^ 1] = *rin;
        return;
    }
    // What the gathers read, double buffered by parity in the handle's m or
    // w vector and the second buffer: w (constant diagonal: m is formed in
    // the gathers and never stored) or m.
    const bool wg = d.dinv_const != 0;
    double *const v0 = (double *)(wg ? d.w : d.m), *const v1 = (double *)d.w1;
    const double *gin = par ? v1 : v0;
    double *gout = par ? v0 : v1;
    const double *tab = nullptr;
    if (vt) {
        if (tid < d.nvtab)
            vtab[tid] = tv;
        __syncthreads();
        tab = vtab;
    }
    PPCG_AS1 double *__restrict__ X = as_global((double *)d.x);
    PPCG_AS1 double *__restrict__ Rv = as_global((double *)d.r);
    // w is read and written in place when it is not what the gathers read
    const PPCG_AS1 double *__restrict__ W = as_global(wg ? gin : (const double *)d.w);
    PPCG_AS1 double *__restrict__ Wo = as_global(wg ? gout : (double *)d.w);
    PPCG_AS1 double *__restrict__ M = as_global(gout);
    PPCG_AS1 double *__restrict__ Z = as_global((double *)d.z);
    PPCG_AS1 double *__restrict__ S = as_global((double *)d.s);
    PPCG_AS1 double *__restrict__ P = as_global((double *)d.p);
    const PPCG_AS1 double *__restrict__ DI = as_global((const double *)d.dinv);
#if PPCG_FUSED_ROW0_EARLY
    // 0. This thread's first row: n = A m_i.
    double nv0 = 0.0;
    {
        const int chunk = row0 / kSellC + wave;
        if (chunk * kSellC < n) {  // uniform per wavefront
            const int64_t eb = lane_i64(ext, 0);
            const int el = (int)((lane_i64(ext, 1) - eb) / kSellC);
            nv0 = fused_row(d, gin, chunk, lane, tab, eb, el, __builtin_amdgcn_readlane(pst, 32));
        }
    }
#endif
    // 1. The previous launch's partials, all tiles of the system, in tile
    // order per thread, then the fixed workgroup tree; the scalar recurrences.
    {
        double v[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
        if (has0) {
            v[0] = v[0] + pa0[0];
            v[1] = v[1] + pa0[1];
            v[2] = v[2] + pb0[0];
            v[3] = v[3] + pb0[1];
        }
        if (has1) {
            v[0] = v[0] + pa1[0];
            v[1] = v[1] + pa1[1];
            v[2] = v[2] + pb1[0];
            v[3] = v[3] + pb1[1];
        }
        for (int t = tid + 2 * kFusedThreads; t < nft; t += kFusedThreads) {
            const dvec2 a = PR[2 * t], b = PR[2 * t + 1];
            v[0] = v[0] + a[0];
            v[1] = v[1] + a[1];
            v[2] = v[2] + b[0];
            v[3] = v[3] + b[1];
        }
        block_sum<kFusedThreads, kNumPartials>(v, lds);
        if (tid == 0) {
            SysState loc = *rin;
            // the update of the previous launch deferred or applied an x-update
            if (!loc.phase) {
                loc.alpha_x = loc.alpha;
                loc.x_pending ^= 1;
            }
            scalar_update<kNumPartials>(d, &loc, v);
            sc.alpha = loc.alpha;
            sc.beta = loc.beta;
            sc.alpha_x = loc.alpha_x;
            sc.x_pending = loc.x_pending;
            sc.go = !loc.done;
            // a stopping system gets its deferred x-update in this launch,
            // so that x is complete when the host reads the state
            sc.x_finish = loc.done && loc.x_pending;
            if (sc.x_finish)
                loc.x_pending = 0;
            if (wi.tile == 0) {
                d.frec[par ^ 1] = loc;
                *d.st = loc;
            }
        }
        __syncthreads();
    }
    if (!sc.go) {
        if (sc.x_finish) {
            const double a = sc.alpha_x;
            for (int k = 0; k < R; ++k) {
                const int i = row0 + k * kFusedThreads + tid;
                if (i < n)
                    X[i] = X[i] + a * P[i];
            }
        }
        return;
    }
    // 2. Per row of this thread (row0 + k * kFusedThreads + tid): n = A m_i
    // into a register, then the fused update with it.
    const double sa = sc.alpha, sb = sc.beta, ax = sc.alpha_x;
    const bool xp = sc.x_pending != 0;
    double acc[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int k = 0; k < R; ++k) {
        const int chunk = (row0 + k * kFusedThreads) / kSellC + wave;
        if (chunk * kSellC >= n)
            break;  // uniform per wavefront: no later chunk of this thread exists either
        const int i = chunk * kSellC + lane;
        const int64_t eb = lane_i64(ext, 2 * k);
        const int el = (int)((lane_i64(ext, 2 * k + 1) - eb) / kSellC);
        const int ep = __builtin_amdgcn_readlane(pst, 32 + k);
#if PPCG_FUSED_ROW0_EARLY
        const double nv = k == 0 ? nv0 : fused_row(d, gin, chunk, lane, tab, eb, el, ep);
#else
        const double nv = fused_row(d, gin, chunk, lane, tab, eb, el, ep);
#endif
        if (i < n) {
            double z = Z[i], w = W[i], s = S[i], p = P[i], r = Rv[i], u, mo;
            const double di = DI[d.dinv_const ? 0 : i];
            const double xo = xp ? X[i] : 0.0;
            const double pold = p;
            vma_elem<double, kNumPartials>(sa, sb, nv, z, w, s, p, r, di, u, mo, acc);
            Z[i] = z;
            S[i] = s;
            P[i] = p;
            Rv[i] = r;
            Wo[i] = w;
            if (!wg)
                M[i] = mo;  // otherwise m_{i+1} = M^-1 w_{i+1} is formed by the next launch's gathers
            if (xp) {
                const double x1 = xo + ax * pold;
                X[i] = x1 + sa * p;
            }
        }
    }
    block_sum<kFusedThreads, kNumPartials>(acc, lds);
    if (tid == 0) {
        PPCG_AS1 dvec2 *out = (PPCG_AS1 dvec2 *)as_global(d.fpart + ((size_t)(par ^ 1) * d.nftiles + wi.tile) * 4);
        out[0] = dvec2{acc[0], acc[1]};
        out[1] = dvec2{acc[2], acc[3]};
    }
}

// First node of every chunk of fused launches (one workgroup per fused
// tile): the canonical state record into slot 0, and after an
// initialisation (phase 1) the initialisation's partials, one record per
// 512-row tile, summed in tile order into one record per fused tile (slot 0).
__global__ void k_fused_begin(const WorkItem *__restrict__ table, const int *__restrict__ count,
                              const SysDesc *__restrict__ descs)
{
    const int pos = blockIdx.x;
    if (pos >= *count)
        return;
    const WorkItem wi = table[pos];
    const SysDesc &d = descs[wi.slot];
    const SysState *st = d.st;
    if (st->done)
        return;
    const int k = threadIdx.x;
    if (st->phase && k < kNumPartials) {
        const int per = d.frows / kTileRows;
        const int t0 = wi.tile * per, t1 = min(t0 + per, d.ntiles);
        const double *src = d.part + (size_t)d.ntiles * kPartStride;  // slot 1
        double a = src[(size_t)t0 * kPartStride + k];
        for (int t = t0 + 1; t < t1; ++t)
            a = a + src[(size_t)t * kPartStride + k];
        d.fpart[(size_t)wi.tile * 4 + k] = a;
    }
    if (wi.tile == 0 && k == 0)
        d.frec[0] = *st;
}

}  // namespace ppcg
