// ppcg_setup.hpp -- device kernels that prepare a matrix (ppcg_create).
//
// Validation and the Jacobi inverse diagonal (Section V-A: Jacobi
// preconditioner, CSR input), then conversion of CSR to SELL-C-sigma: rows
// (optionally sorted by length inside windows of sigma rows) are cut into
// chunks of C = 64, each chunk padded to its longest row and stored
// column-major, so that lane l of a wavefront reads entry k of its row at
// offset k * 64 + l and every load instruction of the wavefront is one
// contiguous 512-byte (values) or 256-byte (columns) segment.
#pragma once

#include "ppcg_internal.hpp"

namespace ppcg {

enum CsrErr : unsigned {
    CSR_E_RP0 = 1u,       // row_ptr[0] != 0
    CSR_E_RPN = 2u,       // row_ptr[n] != nnz
    CSR_E_MONO = 4u,      // row_ptr decreasing or out of [0, nnz]
    CSR_E_COL = 8u,       // column index out of range
    CSR_E_ORDER = 16u,    // columns not strictly ascending in a row
    CSR_E_NODIAG = 32u,   // missing diagonal
    CSR_E_DIAG = 64u,     // diagonal not > 0
    CSR_E_VAL = 128u      // non-finite value
};

// err[0]: OR of CsrErr flags, err[1]: first offending row (atomic min).
__global__ void k_validate(int n, int64_t nnz, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ val, double *__restrict__ dinv, int *__restrict__ rowlen,
                           unsigned *__restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (rp[0] != 0)
            atomicOr(&err[0], CSR_E_RP0);
        if ((int64_t)rp[n] != nnz)
            atomicOr(&err[0], CSR_E_RPN);
    }
    if (i >= n)
        return;
    const int a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || (int64_t)b > nnz) {
        atomicOr(&err[0], CSR_E_MONO);
        atomicMin(&err[1], (unsigned)i);
        rowlen[i] = 0;
        dinv[i] = 0.0;
        return;
    }
    unsigned f = 0;
    int prev = -1;
    double dg = 0.0;
    bool found = false;
    for (int k = a; k < b; ++k) {
        const int c = ci[k];
        const double v = val[k];
        if (c < 0 || c >= n)
            f |= CSR_E_COL;
        else if (c <= prev)
            f |= CSR_E_ORDER;
        prev = c;
        if (!isfinite(v))
            f |= CSR_E_VAL;
        if (c == i) {
            dg = v;
            found = true;
        }
    }
    if (!found)
        f |= CSR_E_NODIAG;
    else if (!(dg > 0.0))
        f |= CSR_E_DIAG;
    if (f) {
        atomicOr(&err[0], f);
        atomicMin(&err[1], (unsigned)i);
    }
    dinv[i] = found && dg > 0.0 ? 1.0 / dg : 0.0;
    rowlen[i] = b - a;
}

// Sort the rows of each window of W rows by decreasing length (ties by
// increasing index): perm[p] = original row at sorted position p.  One
// workgroup per window, bitonic sort of W keys in LDS.
template <int W>
__global__ __launch_bounds__(W / 2 < 512 ? W / 2 : 512) void k_sort_window(int n, const int *__restrict__ rowlen,
                                                                           int *__restrict__ perm)
{
    __shared__ unsigned long long key[W];
    const int w0 = blockIdx.x * W;
    for (int j = threadIdx.x; j < W; j += blockDim.x) {
        const int r = w0 + j;
        key[j] = r < n ? ((unsigned long long)(0xFFFFFFFFu - (unsigned)rowlen[r]) << 32) | (unsigned)j
                       : ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= W; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < W; t += blockDim.x) {
                const int partner = t ^ j;
                if (partner > t) {
                    const bool up = (t & k) == 0;
                    const unsigned long long a = key[t], b = key[partner];
                    if ((a > b) == up) {
                        key[t] = b;
                        key[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < W; j += blockDim.x) {
        const int p = w0 + j;
        if (p < n)
            perm[p] = w0 + (int)(key[j] & 0xFFFFFFFFull);
    }
}

// Sorting windows the autotuner tries (sigma of SELL-C-sigma).
constexpr int kSortWindows[] = {128, 1024, 4096};

// perm for windows of sigma rows (one of kSortWindows).
inline void launch_sort_window(hipStream_t s, int n, int sigma, const int *rowlen, int *perm)
{
    auto grid = [&](int w) { return (unsigned)((n + w - 1) / w); };
    if (sigma == 128)
        k_sort_window<128><<<grid(128), 64, 0, s>>>(n, rowlen, perm);
    else if (sigma == 4096)
        k_sort_window<4096><<<grid(4096), 512, 0, s>>>(n, rowlen, perm);
    else
        k_sort_window<1024><<<grid(1024), 512, 0, s>>>(n, rowlen, perm);
}

__global__ void k_invert_perm(int n, const int *__restrict__ perm, int *__restrict__ invperm)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n)
        invperm[perm[p]] = p;
}

// Entries stored by each chunk: 64 x (longest row of the chunk).
__global__ void k_chunk_size(int n, int nchunks, const int *__restrict__ perm, const int *__restrict__ rowlen,
                             int64_t *__restrict__ sz)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunks)
        return;
    int mx = 0;
    for (int l = 0; l < kSellC; ++l) {
        const int p = c * kSellC + l;
        if (p < n) {
            const int r = perm ? perm[p] : p;
            mx = max(mx, rowlen[r]);
        }
    }
    sz[c] = (int64_t)mx * kSellC;
}

// Exclusive scan of sz[0..m) into out[0..m], single workgroup of 1024.
__global__ __launch_bounds__(1024) void k_scan(int m, const int64_t *__restrict__ sz, int64_t *__restrict__ out)
{
    __shared__ int64_t s[1024];
    const int t = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int a = min(t * per, m), b = min(a + per, m);
    int64_t sum = 0;
    for (int i = a; i < b; ++i)
        sum += sz[i];
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    int64_t run = t ? s[t - 1] : 0;
    for (int i = a; i < b; ++i) {
        out[i] = run;
        run += sz[i];
    }
    if (t == 1023)
        out[m] = s[1023];
}

// Fill SELL arrays.  Stored row p (original row perm[p]) keeps its entries
// in their CSR order; columns are relabelled to sorted positions when the
// rows are permuted.  Padding entries have value 0 and a valid column (the
// row's own position, or n-1 for the rows past n of the last chunk).
__global__ void k_sell_fill(int n, int nchunks, const int *__restrict__ rp, const int *__restrict__ ci,
                            const double *__restrict__ val, const int *__restrict__ perm,
                            const int *__restrict__ invperm, const int64_t *__restrict__ cptr,
                            int *__restrict__ scol, double *__restrict__ sval)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nchunks * kSellC)
        return;
    const int c = p / kSellC, l = p % kSellC;
    const int64_t base = cptr[c];
    const int len = (int)((cptr[c + 1] - base) / kSellC);
    int a = 0, L = 0;
    if (p < n) {
        const int r = perm ? perm[p] : p;
        a = rp[r];
        L = rp[r + 1] - a;
    }
    const int pad_col = p < n ? p : n - 1;
    for (int k = 0; k < len; ++k) {
        const size_t o = (size_t)base + (size_t)k * kSellC + l;
        if (k < L) {
            const int cc = ci[a + k];
            scol[o] = invperm ? invperm[cc] : cc;
            sval[o] = val[a + k];
        } else {
            scol[o] = pad_col;
            sval[o] = 0.0;
        }
    }
}

// Chunk-shared column offsets (stencil-like matrices, rows in their own
// order).  The offsets col - row of a chunk's 64 rows, merged, form its
// shared list; the chunk is stored with that many slots (at least its
// longest row; more where rows of different kinds meet, e.g. the last grid
// line of one plane and the first of the next), entry k of every row at
// offset list[k] from the row, with a zero wherever the row has no entry
// there.  A row's entries keep their ascending column order, so its products
// are added in the order of its CSR entries, with exact zeros in between.
//
// Both kernels run one wavefront per chunk (blockDim 64) and merge the
// rows' offset lists (each ascending, as validated) by repeated minimum.
// k_sell_union_count: cnt[c] = the merged list's length, or -1 when it
// exceeds cap(len) = 2 len + 2 for the chunk's longest row len (then the
// matrix is not stored this way).
__device__ __forceinline__ int wave_min_i32(int m)
{
#pragma unroll
    for (int s = 32; s > 0; s >>= 1)
        m = min(m, __shfl_xor(m, s, 64));
    return m;
}

__global__ __launch_bounds__(64) void k_sell_union_count(int n, int nchunks, const int *__restrict__ rp,
                                                         const int *__restrict__ ci, const int64_t *__restrict__ sz,
                                                         int *__restrict__ cnt)
{
    const int c = blockIdx.x, l = threadIdx.x;
    if (c >= nchunks)
        return;
    const int p = c * kSellC + l;
    const int len = (int)(sz[c] / kSellC);
    int a = 0, L = 0, h = 0;
    if (p < n) {
        a = rp[p];
        L = rp[p + 1] - a;
    }
    const int cap = 2 * len + 2;
    int k = 0;
    for (; k <= cap; ++k) {
        const int off = h < L ? ci[a + h] - p : INT_MAX;
        const int m = wave_min_i32(off);
        if (m == INT_MAX)
            break;
        if (off == m)
            ++h;
    }
    if (l == 0)
        cnt[c] = k > cap ? -1 : k;
}

// k_sell_union: the merged list of chunk c (len = its stored slots, from
// cptr) at lists[cptr[c] / 64 ..], slots past the merged length set to 0;
// flag[0] |= 1 if some row has entries left after len slots.
__global__ __launch_bounds__(64) void k_sell_union(int n, int nchunks, const int *__restrict__ rp,
                                                   const int *__restrict__ ci, const int64_t *__restrict__ cptr,
                                                   int *__restrict__ lists, unsigned *__restrict__ flag)
{
    const int c = blockIdx.x, l = threadIdx.x;
    if (c >= nchunks)
        return;
    const int p = c * kSellC + l;
    const int64_t base = cptr[c];
    const int len = (int)((cptr[c + 1] - base) / kSellC);
    int a = 0, L = 0, h = 0;
    if (p < n) {
        a = rp[p];
        L = rp[p + 1] - a;
    }
    int *out = lists + base / kSellC;
    for (int k = 0; k < len; ++k) {
        const int off = h < L ? ci[a + h] - p : INT_MAX;
        const int m = wave_min_i32(off);
        // (a slot past the merged length repeats the last offset: the list
        // stays ascending, and such a slot holds zeros)
        if (l == 0)
            out[k] = m != INT_MAX ? m : k > 0 ? out[k - 1] : 0;
        if (off == m && m != INT_MAX)
            ++h;
    }
    if (h < L)
        atomicOr(flag, 1u);
}

// Fill the SELL arrays on the chunks' shared offset lists: entry k of row p
// is the row's entry at column p + list[k] when it has one, else value 0 at
// that column clamped into [0, n - 1].  Sets flag[0] |= 1 if an entry of the
// row found no place (cannot happen after k_sell_union succeeded).
__global__ void k_sell_fill_shared(int n, int nchunks, const int *__restrict__ rp, const int *__restrict__ ci,
                                   const double *__restrict__ val, const int64_t *__restrict__ cptr,
                                   const int *__restrict__ cpat, const int *__restrict__ pats,
                                   int *__restrict__ scol, double *__restrict__ sval, unsigned *__restrict__ flag)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nchunks * kSellC)
        return;
    const int c = p / kSellC, l = p % kSellC;
    const int64_t base = cptr[c];
    const int len = (int)((cptr[c + 1] - base) / kSellC);
    const int *list = pats + cpat[c];
    int a = 0, L = 0, h = 0;
    if (p < n) {
        a = rp[p];
        L = rp[p + 1] - a;
    }
    for (int k = 0; k < len; ++k) {
        const size_t o = (size_t)base + (size_t)k * kSellC + l;
        const int t = p + list[k];
        if (h < L && ci[a + h] == t) {
            scol[o] = t;
            sval[o] = val[a + h];
            ++h;
        } else {
            scol[o] = min(max(t, 0), n - 1);
            sval[o] = 0.0;
        }
    }
    if (h < L)
        atomicOr(flag, 1u);
}

// Permute the inverse diagonal into stored-row order.
__global__ void k_permute_d(int n, const int *__restrict__ perm, const double *__restrict__ in,
                            double *__restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n)
        out[p] = in[perm ? perm[p] : p];
}

template <typename TO, typename TI>
__global__ void k_convert(size_t m, const TI *__restrict__ in, TO *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        out[i] = (TO)in[i];
}

}  // namespace ppcg

namespace ppcg {

// flag[0] |= 1 when some dinv[i] differs from dinv[0] (bitwise compare).
__global__ void k_const_check(int n, const double *__restrict__ dinv, unsigned *__restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && __double_as_longlong(dinv[i]) != __double_as_longlong(dinv[0]))
        atomicOr(flag, 1u);
}

}  // namespace ppcg

namespace ppcg {

// SELL column indices as 16-bit offsets from the (stored) row, d = col - row,
// laid out so that a lane reads two of its entries with one dword load: in a
// chunk of padded length len (base = cptr[c], in 16-bit units), entries 2j
// and 2j + 1 of lane l sit at base + 128 j + 2 l and base + 128 j + 2 l + 1;
// when len is odd the last entry sits at base + 128 (len / 2) + l.  A chunk
// still takes 64 len slots, and base is a multiple of 64, so the pair dwords
// are aligned.  flag[0] |= 1 when some offset does not fit 16 bits.
__global__ void k_sell_delta16(int nchunks, const int64_t *__restrict__ cptr, const int *__restrict__ col,
                               short *__restrict__ col16, unsigned *__restrict__ flag)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nchunks * kSellC)
        return;
    const int c = p / kSellC, l = p % kSellC;
    const int row = c * kSellC + l;
    const int64_t base = cptr[c];
    const int len = (int)((cptr[c + 1] - base) / kSellC);
    const int paired = len & ~1;
    bool ok = true;
    for (int k = 0; k < len; ++k) {
        const size_t o = (size_t)base + (size_t)k * kSellC + l;
        const int d = col[o] - row;
        ok = ok && d >= -32768 && d <= 32767;
        const size_t dst = k < paired ? (size_t)base + (size_t)(k >> 1) * (2 * kSellC) + 2 * l + (k & 1)
                                      : (size_t)base + (size_t)paired * kSellC + l;
        col16[dst] = (short)d;
    }
    if (!ok)
        atomicOr(flag, 1u);
}

// One-byte value indices: vidx[e] = the position of the stored value val[e]
// in tab, the matrix's distinct values as ascending unsigned 64-bit bit
// patterns (ntab in [1, kMaxValueTable]), found by binary search.  A value
// missing from the table sets flag[0] |= 1 (and index 0); the caller then
// drops the indices.
__global__ void k_sell_vidx(int64_t stored, const double *__restrict__ val, const unsigned long long *__restrict__ tab,
                            int ntab, unsigned char *__restrict__ vidx, unsigned *__restrict__ flag)
{
    __shared__ unsigned long long t[kMaxValueTable];
    for (int k = threadIdx.x; k < ntab; k += blockDim.x)
        t[k] = tab[k];
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= stored)
        return;
    const unsigned long long key = (unsigned long long)__double_as_longlong(val[e]);
    int lo = 0, hi = ntab - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (t[lo] != key) {
        atomicOr(flag, 1u);
        lo = 0;
    }
    vidx[e] = (unsigned char)lo;
}

}  // namespace ppcg
