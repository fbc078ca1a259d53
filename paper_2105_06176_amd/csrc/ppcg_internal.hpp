// ppcg_internal.hpp -- data structures shared by the HIP kernels and the host
// runtime of the PIPECG library.
//
// Work decomposition.  Every system (one handle) is cut into tiles of
// kTileRows consecutive rows.  A launch processes a table of work items
// (system slot, tile index); one workgroup handles one work item.  A single
// solve is a table over one system, a batched solve a table over many, and
// the arithmetic a system sees does not depend on what else is in the table:
// its tiles, their per-tile partial sums and the fixed-order reduction of
// those partials are the same alone and in a mix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

namespace ppcg {

constexpr int kTileRows = 512;     // rows per work item (both kernels)
constexpr int kVmaThreads = 256;   // fused update kernel: 2 rows per thread
constexpr int kSpmvThreads = 512;  // SpMV kernel: 8 wavefronts, one row per lane (SELL)
constexpr int kSellC = 64;         // SELL chunk height = wavefront width
constexpr int kSellChunksPerTile = kTileRows / kSellC;
constexpr int kSortWindow = 1024;  // SELL sigma when sorting is used
constexpr int kNumPartials = 4;    // (r,u), (w,u), (u,u), (r,r)
constexpr int kPartStride = 8;     // doubles per tile partial record (replacement uses 6)
// The single-launch iteration (ppcg_fused.hpp): tiles of kFusedRows rows,
// kFusedRowsPerThread rows per thread.
#ifndef PPCG_FUSED_THREADS
#define PPCG_FUSED_THREADS 512
#endif
#ifndef PPCG_FUSED_ROWS_PER_THREAD
#define PPCG_FUSED_ROWS_PER_THREAD 16
#endif
constexpr int kFusedThreads = PPCG_FUSED_THREADS;
constexpr int kFusedRowsPerThread = PPCG_FUSED_ROWS_PER_THREAD;  // at most
constexpr int kFusedRows = kFusedThreads * kFusedRowsPerThread;    // at most
static_assert(kFusedThreads == kTileRows, "a fused tile is a whole number of 512-row tiles");
// Workgroups of the single-launch kernel one compute unit holds at once (its
// 76 VGPRs allow 6 wavefronts per SIMD: 3 workgroups of 8 wavefronts).
constexpr int kFusedResidentPerCU = 3;

// Rows per fused tile (R rows per thread) for a system of n rows on a GPU of
// `cus` compute units.  The smallest candidate keeps the tile count at or
// below 256 (at most 4 rows per thread), so that a small system still spreads
// over many workgroups while every workgroup re-reads few partial-sum
// records (one per tile).  Larger R (up to kFusedRowsPerThread) is taken
// when it shortens the launch by the model below.
//
// Model: a compute unit gets w = ceil(tiles / cus) workgroups and holds
// kFusedResidentPerCU at once.  With w at most that, its time is w tiles of
// R rows; beyond it, its workgroups run in ceil(w / 3) rounds of 3, each round
// costing as much as a full one (the last, partly filled round runs at low
// occupancy).  Cost = R * w, or R * 3 * ceil(w / 3); the smallest R wins
// ties.  Measured (us per iteration, 16-bit columns and value table):
// 128^3 (2,097,152 rows) R = 8 (512 tiles) 51.9 against R = 4 55.0 and
// R = 6 56.1; 2048^2 (4,194,304 rows) R = 16 (512 tiles) 91.4 against R = 4
// 95.6 and R = 8 101.3; 160^3 7-point R = 16 94.1 against R = 4 98.0.
#ifndef PPCG_FUSED_TILE_TARGET
#define PPCG_FUSED_TILE_TARGET 256
#endif
inline int fused_tile_rows(int n, int cus)
{
    constexpr int kTarget = PPCG_FUSED_TILE_TARGET;
    int r0 = (n + kTarget * kFusedThreads - 1) / (kTarget * kFusedThreads);
    r0 = r0 < 1 ? 1 : r0 > 4 ? 4 : r0;
    if (cus < 1)
        cus = 1;
    int best = r0;
    long long best_cost = -1;
    for (int r = r0; r <= kFusedRowsPerThread; ++r) {
        const long long rows = (long long)r * kFusedThreads;
        const long long tiles = (n + rows - 1) / rows;
        const long long w = (tiles + cus - 1) / cus;
        const long long cost = w <= kFusedResidentPerCU
                                   ? r * w
                                   : r * kFusedResidentPerCU * ((w + kFusedResidentPerCU - 1) / kFusedResidentPerCU);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = r;
        }
    }
    return best * kFusedThreads;
}
static_assert(kFusedThreads % kSellC == 0, "each wavefront of a fused tile reads whole SELL chunks");

// Tile-to-workgroup mapping.  The fused update is a pure stream and runs
// slightly faster with each XCD owning a contiguous range of tiles; the SpMV
// measured slightly faster with the plain round-robin mapping.
#ifndef PPCG_XCD_REMAP
#define PPCG_XCD_REMAP 1
#endif
#ifndef PPCG_XCD_REMAP_SPMV
#define PPCG_XCD_REMAP_SPMV 0
#endif

#ifndef PPCG_SELL_VTAB
#define PPCG_SELL_VTAB 1  // one-byte value indices into a table of distinct values, when timed faster
#endif
// 1: rows in their own order are stored on chunk-shared offset lists when
// every chunk has one, and the FP64 PIPECG SpMV reads the lists instead of a
// column per entry when that timed faster (0: never).
#ifndef PPCG_SELL_SHARED
#define PPCG_SELL_SHARED 1
#endif
// Entries per straight span on shared offset lists.  16 would put more
// gathers in flight per wavefront, but takes the single-launch kernel from
// 74 to 105 VGPRs (4 wavefronts per SIMD instead of 6) and spills in the SpMV.
#ifndef PPCG_SHARED_BATCH
#define PPCG_SHARED_BATCH 8
#endif
// 1: for SELL matrices whose column offsets from the row fit 16 bits, time
// the SpMV with 16-bit offsets against 32-bit columns at setup and keep the
// faster (0: 32-bit columns only).
#ifndef PPCG_SELL_COL16
#define PPCG_SELL_COL16 1
#endif

// SELL SpMV: entries per lane whose column and value loads are issued
// together before their gathers (even: the 16-bit layout reads pairs).
#ifndef PPCG_SELL_BATCH
#define PPCG_SELL_BATCH 8
#endif
// 1: the 16-bit-column SELL rows overlap the next batch's loads with the
// current batch's gathers (27-point 160^3: 245.1 -> 241.6 us per SpMV).
#ifndef PPCG_SELL_PIPE
#define PPCG_SELL_PIPE 1
#endif
// 1: SELL rows with 16-bit columns or the one-byte value table as straight
// spans of loads with no per-entry branch (sell_row_straight); 0: the
// guarded batch loop.  On the single-launch iteration: 128^3 7-point with
// both, 90.9 -> 57.6 us; 2048^2 5-point, 147 -> 109 us.
#ifndef PPCG_SELL_STRAIGHT
#define PPCG_SELL_STRAIGHT 1
#endif
// 1: also the rows of 32-bit columns with 8-byte values whose gathers scale
// w into m (the single-launch iteration with a constant diagonal) run as
// straight spans: 128^3, 78.5 -> 66.7 us per iteration.
// 1: the classic-PCG SpMV with FP32 values and FP64 vectors also reads the
// 16-bit column offsets (0: 32-bit columns for that combination; the 27-point 160^3
// solve with them, straight spans in both: 210.9 against 207.0 ms).
#ifndef PPCG_PCG_V32_COL16
#define PPCG_PCG_V32_COL16 0
#endif
#ifndef PPCG_SELL_STRAIGHT_SC
#define PPCG_SELL_STRAIGHT_SC 1
#endif
#ifndef PPCG_SELL_PIPE_BATCH
#define PPCG_SELL_PIPE_BATCH 4
#endif
// Waves per SIMD the SpMV is compiled for (8: at most 64 VGPRs).
#ifndef PPCG_SPMV_WAVES
#define PPCG_SPMV_WAVES 8
#endif

// Systems with at most this many rows (SELL format, FP64) iterate in the
// one-workgroup kernel: for them launch latency, not bandwidth, dominates.
#ifndef PPCG_SMALL_MAX_ROWS
#define PPCG_SMALL_MAX_ROWS 4096
#endif

enum Fmt : int { FMT_SELL = 1, FMT_CSRV = 2 };
enum Prec : int { PREC_F64 = 0, PREC_F32 = 1, PREC_V32 = 2 /* FP32 values, FP64 vectors */ };

// Status codes mirrored from ppcg.h (device code does not include it).
enum DevStatus : int {
    ST_OK = 0,
    ST_NOT_CONVERGED = 1,
    ST_BREAKDOWN = 2,
    ST_STAGNATED = 3,
    ST_REPLACE = 4  // FP32-values mode: paused for a reliable update (not a final status)
};
enum StopMode : int { STOP_REL = 0, STOP_ABS = 1 };

// Per-system iteration state.  Lives in device memory, written only by the
// designated workgroup of the SpMV launch (or by the start kernel), read by
// every workgroup; mirrored to pinned host memory for polling.
struct alignas(128) SysState {
    double gamma;       // (r_i, u_i)
    double delta;       // (w_i, u_i)
    double uu;          // (u_i, u_i)
    double rr;          // (r_i, r_i)
    double alpha;       // alpha_i used by the next fused update
    double beta;        // beta_i used by the next fused update
    double gamma_prev;  // gamma_{i-1}
    double alpha_prev;  // alpha_{i-1}
    double gamma_prev2; // gamma_{i-1} as it was before the last scalar update
    double repl_ref;    // FP32-values mode: residual norm at the last start / reliable update
    double bnorm2;      // (b, b)
    double tnorm2;      // (b - A x, b - A x) from the last true-residual pass
    double alpha_x;     // alpha of the x-update the fused update deferred (x_pending)
    int iter;           // x-updates so far (all starts)
    int i_start;        // x-updates in the current start
    int done;           // 1: stop iterating
    int status;         // DevStatus when done
    int phase;          // 1: the next reduction is the one that ends initialisation
    int x_pending;      // 1: x still lacks alpha_x * p (the fused update defers every other x-update)
};
static_assert(sizeof(SysState) == 128, "SysState is one 128-byte record");

// Per-system descriptor (device-resident copy per engine slot).
// Largest value table: a one-byte index per stored entry.
constexpr int kMaxValueTable = 256;
// Longest concatenation of distinct shared offset lists kept (ints): the
// lists are read through the scalar cache, so only a few KB of them are used.
constexpr int kMaxSharedOffsets = 8192;

struct SysDesc {
    int n;
    int ntiles;
    int fmt;            // Fmt
    int lanes;          // CSR-vector lanes per row
    int stop;           // StopMode
    int maxit;
    int fixed;          // > 0: fixed number of iterations
    int prec;           // Prec of the vectors and values below
    int pair;           // mixed precision: slot of the same system in the other group
    int vals32;         // 1: iteration SpMVs read the FP32 copy of the values (val32)
    int dinv_const;     // 1: every diagonal entry is equal; the updates read dinv[0] for every row
    int nvtab;          // entries of vtab (when vidx is set)
    double tol;
    double repl_factor; // vals32: pause for a reliable update when the residual fell by this factor
    const int64_t *cptr;  // SELL chunk offsets [nchunks + 1]
    const int *rp;        // CSR row pointers [n + 1] (CSR-vector format)
    const int *col;       // SELL / CSR column indices
    const short *col16;   // SELL: column minus row as 16-bit offsets when every one fits (else NULL)
    const unsigned char *vidx;  // SELL, FP64 values: index of each stored value in vtab (else NULL)
    const double *vtab;   // the matrix's distinct values (at most kMaxValueTable), ascending bit patterns
    const int *cpat;      // SELL: start of each chunk's shared offset list in pats, when the FP64
                          // PIPECG SpMV reads them (else NULL)
    const int *pats;      // the distinct offset lists, concatenated
    const void *val;      // matrix values (double or float)
    const float *val32;   // FP32 copy of the values (vals32 mode)
    const void *dinv;     // inverse diagonal (double or float)
    void *x, *r, *u, *w, *m, *nv, *z, *q, *s, *p;  // solver vectors
    const void *b;        // right-hand side (internal copy)
    double *part;         // partial sums: 2 slots x ntiles x kPartStride
    SysState *st;
    // single-launch iteration (ppcg_fused.hpp); unused by the two-launch form
    int nftiles;          // fused tiles (of frows rows)
    int frows;            // rows per fused tile (fused_tile_rows(n, compute units))
    SysState *frec;       // scalar state, 2 slots (launch parity)
    double *fpart;        // partial sums, 2 slots x nftiles x 4
    void *w1;             // second buffer of what the gathers read (w, or m for a diagonal that is not
                          // constant), which every tile reads while it is being rewritten
};

struct WorkItem {
    int slot;  // index into the engine's SysDesc array
    int tile;  // tile index within that system
};

}  // namespace ppcg
