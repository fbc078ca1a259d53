// ppcg_shard.hip -- the row split of the performance model and one unit's
// share of A under the 2-D decomposition (Tiwari & Vadhiyar, Section IV-C,
// "Performance Modelling" and "Data Decomposition"), with its two-part SpMV.
//
// A unit owns the rows [lo, hi).  Its entries are split by column: part 1
// holds the entries whose column is also in [lo, hi) (they need only the
// unit's own piece of the input vector), part 2 the others, whose columns
// are renumbered to a compact halo vector listing the distinct remote
// columns in ascending order.  Part 1 runs while the halo is in transit;
// part 2 completes the product once it has arrived.  Both parts are stored
// SELL-C (C = 64, one lane per row, no sorting); part 2 only over the rows
// that have remote entries (boundary rows).  Each row sums its part-1 and
// its part-2 entries separately in stored column order and adds the two.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "ppcg_engine.hpp"

using namespace ppcg;

namespace {

constexpr int kShardThreads = 512;  // 8 wavefronts = 8 SELL chunks per workgroup

struct HostSell {
    int rows = 0;
    int nchunks = 0;
    std::vector<int64_t> cptr;
    std::vector<int> col;
    std::vector<double> val;
};

// SELL-C of the given rows; entries[r] = (column, value) pairs in stored order.
HostSell build_host_sell(const std::vector<std::vector<std::pair<int, double>>> &entries, int pad_col_base,
                         bool pad_own_row)
{
    HostSell s;
    s.rows = (int)entries.size();
    s.nchunks = (s.rows + kSellC - 1) / kSellC;
    s.cptr.assign(s.nchunks + 1, 0);
    for (int c = 0; c < s.nchunks; ++c) {
        size_t len = 0;
        for (int l = 0; l < kSellC && c * kSellC + l < s.rows; ++l)
            len = std::max(len, entries[c * kSellC + l].size());
        s.cptr[c + 1] = s.cptr[c] + (int64_t)len * kSellC;
    }
    s.col.assign(s.cptr[s.nchunks], 0);
    s.val.assign(s.cptr[s.nchunks], 0.0);
    for (int c = 0; c < s.nchunks; ++c) {
        const int64_t base = s.cptr[c];
        const int len = (int)((s.cptr[c + 1] - base) / kSellC);
        for (int l = 0; l < kSellC; ++l) {
            const int r = c * kSellC + l;
            const int pad = pad_own_row && r < s.rows ? r : pad_col_base;
            for (int k = 0; k < len; ++k) {
                const size_t o = (size_t)base + (size_t)k * kSellC + l;
                if (r < s.rows && k < (int)entries[r].size()) {
                    s.col[o] = entries[r][k].first;
                    s.val[o] = entries[r][k].second;
                } else {
                    s.col[o] = pad;  // zero value: adds nothing
                }
            }
        }
    }
    return s;
}

// One SELL-C row (chunk, lane): entry k at cptr[chunk] + k * 64 + lane, summed
// in stored order; entries are fetched in batches of 8 (column indices and
// values first, then the gathers) so each lane keeps several loads in flight.
// The chunk length is uniform across the wavefront, so the guards do not
// diverge.
__device__ __forceinline__ double shard_row(const int64_t *__restrict__ cptr, const int *__restrict__ col,
                                            const double *__restrict__ val, const double *__restrict__ x,
                                            int chunk, int lane)
{
    constexpr int B = 8;
    const int64_t base = cptr[chunk];
    const int len = (int)((cptr[chunk + 1] - base) / kSellC);
    const int *c = col + base + lane;
    const double *v = val + base + lane;
    double acc = 0.0;
    for (int k0 = 0; k0 < len; k0 += B) {
        int cc[B];
        double vv[B], xx[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            cc[j] = 0;
            vv[j] = 0.0;
            if (k0 + j < len) {
                cc[j] = __builtin_nontemporal_load(c + (size_t)(k0 + j) * kSellC);
                vv[j] = __builtin_nontemporal_load(v + (size_t)(k0 + j) * kSellC);
            }
        }
#pragma unroll
        for (int j = 0; j < B; ++j)
            xx[j] = k0 + j < len ? x[cc[j]] : 0.0;
#pragma unroll
        for (int j = 0; j < B; ++j)
            if (k0 + j < len)
                acc = acc + vv[j] * xx[j];
    }
    return acc;
}

// Part 1: y[i] = sum of the row's local entries (x indexed by local row).
__global__ __launch_bounds__(kShardThreads) void k_shard_part1(int rows, const int64_t *__restrict__ cptr,
                                                               const int *__restrict__ col,
                                                               const double *__restrict__ val,
                                                               const double *__restrict__ x, double *__restrict__ y)
{
    const int chunk = blockIdx.x * (kShardThreads / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (chunk * kSellC >= rows)
        return;
    const double acc = shard_row(cptr, col, val, x, chunk, lane);
    const int i = chunk * kSellC + lane;
    if (i < rows)
        y[i] = acc;
}

// Part 2: y[brow[b]] += sum of boundary row b's remote entries (halo indexed).
__global__ __launch_bounds__(kShardThreads) void k_shard_part2(int nb, const int *__restrict__ brow,
                                                               const int64_t *__restrict__ cptr,
                                                               const int *__restrict__ col,
                                                               const double *__restrict__ val,
                                                               const double *__restrict__ xh, double *__restrict__ y)
{
    const int chunk = blockIdx.x * (kShardThreads / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (chunk * kSellC >= nb)
        return;
    const double acc = shard_row(cptr, col, val, xh, chunk, lane);
    const int b = chunk * kSellC + lane;
    if (b < nb) {
        const int i = brow[b];
        y[i] = y[i] + acc;
    }
}

// Halo receive on one device: xh[k] = x[cols[k]] from the global vector.
__global__ void k_shard_gather(int h, const int *__restrict__ cols, const double *__restrict__ x,
                               double *__restrict__ xh)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < h)
        xh[k] = x[cols[k]];
}

}  // namespace

#include "ppcg_shard_internal.hpp"

ppcg_status shard_launch(ppcg_shard *s, int which, const double *x_local, const double *x_halo, double *y,
                         hipEvent_t e0, hipEvent_t e1)
{
    const int rows = s->hi - s->lo;
    const int cpb = kShardThreads / 64;
    if (which == 1) {
        const int grid = (s->nch1 + cpb - 1) / cpb;
        hipExtLaunchKernelGGL(k_shard_part1, dim3(grid), dim3(kShardThreads), 0, s->stream, e0, e1, 0, rows,
                              (const int64_t *)s->cptr1, (const int *)s->col1, (const double *)s->val1, x_local, y);
    } else if (s->nb > 0) {
        const int grid = (s->nch2 + cpb - 1) / cpb;
        hipExtLaunchKernelGGL(k_shard_part2, dim3(grid), dim3(kShardThreads), 0, s->stream, e0, e1, 0, s->nb,
                              (const int *)s->brow, (const int64_t *)s->cptr2, (const int *)s->col2,
                              (const double *)s->val2, x_halo, y);
    }
    PPCG_HIP(hipGetLastError());
    return PPCG_OK;
}

extern "C" {

ppcg_status ppcg_split_rows(int32_t n, const int32_t *row_ptr, int32_t parts, const double *spmv_times,
                            int32_t *row_begin)
{
    clear_error();
    if (n < 1 || !row_ptr || parts < 1 || !spmv_times || !row_begin) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    for (int k = 0; k < parts; ++k)
        if (!(spmv_times[k] > 0.0) || !std::isfinite(spmv_times[k])) {
            set_error("spmv_times[%d] must be finite and > 0", k);
            return PPCG_ERR_INVALID_ARG;
        }
    if (row_ptr[0] != 0) {
        set_error("row_ptr[0] must be 0");
        return PPCG_ERR_BAD_CSR;
    }
    for (int i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) {
            set_error("row_ptr decreases at row %d", i);
            return PPCG_ERR_BAD_CSR;
        }
    const double nnz = (double)row_ptr[n];
    if (nnz == 0.0) {  // no non-zeros to share: the first unit takes every row
        row_begin[0] = 0;
        for (int k = 1; k <= parts; ++k)
            row_begin[k] = n;
        return PPCG_OK;
    }
    // s_k = nnz / t_k, r_k = s_k / sum s (Section IV-C, Performance Modelling)
    std::vector<double> s(parts);
    double tot = 0.0;
    for (int k = 0; k < parts; ++k) {
        s[k] = nnz / spmv_times[k];
        tot += s[k];
    }
    row_begin[0] = 0;
    double cum = 0.0;
    int b = 0;
    for (int k = 0; k + 1 < parts; ++k) {
        cum += s[k] / tot;
        const double target = nnz * cum;
        // most leading rows whose non-zeros number at most the target
        while (b < n && (double)row_ptr[b + 1] <= target)
            ++b;
        row_begin[k + 1] = b;
    }
    row_begin[parts] = n;
    return PPCG_OK;
}

ppcg_status ppcg_shard_destroy(ppcg_shard *s)
{
    clear_error();
    if (!s)
        return PPCG_OK;
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    s->arena.release();
    delete s;
    return PPCG_OK;
}

ppcg_status ppcg_shard_create(const ppcg_csr *A, int32_t row_begin, int32_t row_end, void *hip_stream,
                              ppcg_shard **out)
{
    clear_error();
    if (!out || !A || A->struct_size != sizeof(ppcg_csr) || A->n < 1 || A->nnz < 0 || A->nnz >= INT32_MAX ||
        !A->row_ptr || !A->col_idx || !A->values || (A->mem != PPCG_MEM_HOST && A->mem != PPCG_MEM_DEVICE) ||
        row_begin < 0 || row_end <= row_begin || row_end > A->n) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    const int n = A->n;
    const int64_t nnz = A->nnz;
    // Host view of the CSR (copied from the device when needed).
    std::vector<int32_t> rp_h, ci_h;
    std::vector<double> val_h;
    const int32_t *rp = A->row_ptr, *ci = A->col_idx;
    const double *va = A->values;
    if (A->mem == PPCG_MEM_DEVICE) {
        PPCG_TRY(check_dev_range(A->row_ptr, sizeof(int32_t) * (n + 1), "row_ptr"));
        PPCG_TRY(check_dev_range(A->col_idx, sizeof(int32_t) * nnz, "col_idx"));
        PPCG_TRY(check_dev_range(A->values, sizeof(double) * nnz, "values"));
        rp_h.resize(n + 1);
        ci_h.resize(nnz);
        val_h.resize(nnz);
        PPCG_HIP(hipMemcpy(rp_h.data(), A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
        PPCG_HIP(hipMemcpy(ci_h.data(), A->col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
        PPCG_HIP(hipMemcpy(val_h.data(), A->values, sizeof(double) * nnz, hipMemcpyDeviceToHost));
        rp = rp_h.data();
        ci = ci_h.data();
        va = val_h.data();
    }
    if (rp[0] != 0 || rp[n] != nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[n] = nnz");
        return PPCG_ERR_BAD_CSR;
    }
    const int lo = row_begin, hi = row_end;
    for (int i = lo; i < hi; ++i) {
        if (rp[i + 1] < rp[i]) {
            set_error("row_ptr decreases at row %d", i);
            return PPCG_ERR_BAD_CSR;
        }
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] < 0 || ci[k] >= n || !std::isfinite(va[k])) {
                set_error("row %d: column index out of range or value not finite", i);
                return PPCG_ERR_BAD_CSR;
            }
    }
    std::unique_ptr<ppcg_shard> s(new ppcg_shard());
    PPCG_HIP(hipGetDevice(&s->device));
    s->stream = (hipStream_t)hip_stream;
    s->n = n;
    s->lo = lo;
    s->hi = hi;
    // Distinct remote columns, ascending: the halo.
    std::vector<int> rem;
    for (int i = lo; i < hi; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] < lo || ci[k] >= hi)
                rem.push_back(ci[k]);
    std::sort(rem.begin(), rem.end());
    rem.erase(std::unique(rem.begin(), rem.end()), rem.end());
    s->halo = (int)rem.size();
    s->halo_cols = rem;
    std::vector<std::vector<std::pair<int, double>>> e1(hi - lo), e2;
    std::vector<int> brow;
    for (int i = lo; i < hi; ++i) {
        std::vector<std::pair<int, double>> r2;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int c = ci[k];
            if (c >= lo && c < hi) {
                e1[i - lo].push_back({c - lo, va[k]});
            } else {
                const int slot = (int)(std::lower_bound(rem.begin(), rem.end(), c) - rem.begin());
                r2.push_back({slot, va[k]});
            }
        }
        s->nnz1 += (int64_t)e1[i - lo].size();
        if (!r2.empty()) {
            s->nnz2 += (int64_t)r2.size();
            brow.push_back(i - lo);
            e2.push_back(std::move(r2));
        }
    }
    s->nb = (int)brow.size();
    const HostSell p1 = build_host_sell(e1, 0, true);
    const HostSell p2 = build_host_sell(e2, 0, false);
    s->nch1 = p1.nchunks;
    s->nch2 = p2.nchunks;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bytes = al(sizeof(int64_t) * p1.cptr.size()) + al(sizeof(int) * p1.col.size()) +
                         al(sizeof(double) * p1.val.size()) + al(sizeof(int64_t) * p2.cptr.size()) +
                         al(sizeof(int) * p2.col.size()) + al(sizeof(double) * p2.val.size()) +
                         al(sizeof(int) * brow.size()) + al(sizeof(int) * rem.size()) + 256;
    PPCG_TRY(s->arena.alloc(bytes));
    s->cptr1 = (int64_t *)s->arena.take(sizeof(int64_t) * p1.cptr.size());
    s->col1 = (int *)s->arena.take(sizeof(int) * p1.col.size());
    s->val1 = (double *)s->arena.take(sizeof(double) * p1.val.size());
    s->cptr2 = (int64_t *)s->arena.take(sizeof(int64_t) * p2.cptr.size());
    s->col2 = (int *)s->arena.take(sizeof(int) * p2.col.size());
    s->val2 = (double *)s->arena.take(sizeof(double) * p2.val.size());
    s->brow = (int *)s->arena.take(sizeof(int) * brow.size());
    s->hcols = (int *)s->arena.take(sizeof(int) * rem.size());
    auto up = [&](void *dst, const void *src, size_t b) -> ppcg_status {
        if (b)
            PPCG_HIP(hipMemcpy(dst, src, b, hipMemcpyHostToDevice));
        return PPCG_OK;
    };
    PPCG_TRY(up(s->cptr1, p1.cptr.data(), sizeof(int64_t) * p1.cptr.size()));
    PPCG_TRY(up(s->col1, p1.col.data(), sizeof(int) * p1.col.size()));
    PPCG_TRY(up(s->val1, p1.val.data(), sizeof(double) * p1.val.size()));
    PPCG_TRY(up(s->cptr2, p2.cptr.data(), sizeof(int64_t) * p2.cptr.size()));
    PPCG_TRY(up(s->col2, p2.col.data(), sizeof(int) * p2.col.size()));
    PPCG_TRY(up(s->val2, p2.val.data(), sizeof(double) * p2.val.size()));
    PPCG_TRY(up(s->brow, brow.data(), sizeof(int) * brow.size()));
    PPCG_TRY(up(s->hcols, rem.data(), sizeof(int) * rem.size()));
    *out = s.release();
    return PPCG_OK;
}

ppcg_status ppcg_shard_get_info(const ppcg_shard *s, ppcg_shard_info *info)
{
    clear_error();
    if (!s || !info || info->struct_size != sizeof(ppcg_shard_info)) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    info->row_begin = s->lo;
    info->row_end = s->hi;
    info->nnz_local = s->nnz1;
    info->nnz_remote = s->nnz2;
    info->halo = s->halo;
    info->boundary_rows = s->nb;
    const double rows = s->hi - s->lo;
    // algorithmic bytes: values + columns of every entry, chunk pointers, the
    // input entries once, the output written (part 2: read and written)
    info->bytes_part1 = 12.0 * (double)s->nnz1 + 8.0 * (s->nch1 + 1) + 8.0 * rows + 8.0 * rows;
    info->bytes_part2 = 12.0 * (double)s->nnz2 + 8.0 * (s->nch2 + 1) + 4.0 * s->nb + 8.0 * s->halo +
                        16.0 * s->nb;
    info->halo_bytes = 8.0 * s->halo;
    return PPCG_OK;
}

ppcg_status ppcg_shard_halo_columns(const ppcg_shard *s, int32_t *cols)
{
    clear_error();
    if (!s || (!cols && s->halo > 0)) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    if (s->halo)
        memcpy(cols, s->halo_cols.data(), sizeof(int32_t) * s->halo);
    return PPCG_OK;
}


ppcg_status ppcg_shard_gather(ppcg_shard *s, const double *x_global, double *x_halo)
{
    clear_error();
    if (!s) {
        set_error("shard is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    if (s->halo == 0)
        return PPCG_OK;
    PPCG_HIP(hipSetDevice(s->device));
    PPCG_TRY(check_dev_range(x_global, sizeof(double) * s->n, "x_global"));
    PPCG_TRY(check_dev_range(x_halo, sizeof(double) * s->halo, "x_halo"));
    k_shard_gather<<<(s->halo + 255) / 256, 256, 0, s->stream>>>(s->halo, s->hcols, x_global, x_halo);
    PPCG_HIP(hipGetLastError());
    PPCG_HIP(hipStreamSynchronize(s->stream));
    return PPCG_OK;
}

ppcg_status ppcg_shard_spmv(ppcg_shard *s, const double *x_local, const double *x_halo, double *y, int32_t parts)
{
    clear_error();
    if (!s || parts < 1 || parts > 3) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_HIP(hipSetDevice(s->device));
    const size_t rows = (size_t)(s->hi - s->lo);
    PPCG_TRY(check_dev_range(y, sizeof(double) * rows, "y"));
    if (parts & 1)
        PPCG_TRY(check_dev_range(x_local, sizeof(double) * rows, "x_local"));
    if ((parts & 2) && s->halo > 0)
        PPCG_TRY(check_dev_range(x_halo, sizeof(double) * s->halo, "x_halo"));
    if ((parts & 1) && (const double *)y == x_local) {
        set_error("y must not alias x_local");
        return PPCG_ERR_INVALID_ARG;
    }
    if (parts & 1)
        PPCG_TRY(shard_launch(s, 1, x_local, x_halo, y, nullptr, nullptr));
    if (parts & 2)
        PPCG_TRY(shard_launch(s, 2, x_local, x_halo, y, nullptr, nullptr));
    PPCG_HIP(hipStreamSynchronize(s->stream));
    return PPCG_OK;
}

ppcg_status ppcg_shard_time(ppcg_shard *s, const double *x_global, const double *x_local, double *x_halo, double *y,
                            int32_t iters, double *ms_part1, double *ms_gather, double *ms_part2)
{
    clear_error();
    if (!s || iters < 1 || iters > 10000 || !ms_part1 || !ms_gather || !ms_part2) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_HIP(hipSetDevice(s->device));
    const size_t rows = (size_t)(s->hi - s->lo);
    PPCG_TRY(check_dev_range(y, sizeof(double) * rows, "y"));
    PPCG_TRY(check_dev_range(x_local, sizeof(double) * rows, "x_local"));
    PPCG_TRY(check_dev_range(x_global, sizeof(double) * s->n, "x_global"));
    if (s->halo > 0)
        PPCG_TRY(check_dev_range(x_halo, sizeof(double) * s->halo, "x_halo"));
    std::vector<hipEvent_t> ev(6, nullptr);
    auto clean = [&]() {
        (void)hipStreamSynchronize(s->stream);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            clean();
            set_error("hipEventCreate failed");
            return PPCG_ERR_DEVICE;
        }
    double t1 = 0, tg = 0, t2 = 0;
    for (int it = 0; it < iters; ++it) {
        ppcg_status rc = shard_launch(s, 1, x_local, x_halo, y, ev[0], ev[1]);
        if (rc == PPCG_OK && s->halo > 0) {
            hipExtLaunchKernelGGL(k_shard_gather, dim3((s->halo + 255) / 256), dim3(256), 0, s->stream, ev[2],
                                  ev[3], 0, s->halo, (const int *)s->hcols, x_global, x_halo);
            if (hipGetLastError() != hipSuccess)
                rc = PPCG_ERR_DEVICE;
        }
        if (rc == PPCG_OK && s->nb > 0)
            rc = shard_launch(s, 2, x_local, x_halo, y, ev[4], ev[5]);
        if (rc == PPCG_OK && hipStreamSynchronize(s->stream) != hipSuccess)
            rc = PPCG_ERR_DEVICE;
        if (rc != PPCG_OK) {
            clean();
            return rc;
        }
        float a = 0, g = 0, c = 0;
        (void)hipEventElapsedTime(&a, ev[0], ev[1]);
        if (s->halo > 0)
            (void)hipEventElapsedTime(&g, ev[2], ev[3]);
        if (s->nb > 0)
            (void)hipEventElapsedTime(&c, ev[4], ev[5]);
        t1 += a;
        tg += g;
        t2 += c;
    }
    *ms_part1 = t1 / iters;
    *ms_gather = tg / iters;
    *ms_part2 = t2 / iters;
    clean();
    return PPCG_OK;
}

}  // extern "C"
