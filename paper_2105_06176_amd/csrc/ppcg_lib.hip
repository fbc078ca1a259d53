// ppcg_lib.hip -- the PIPECG library: matrix setup, the iteration engine and
// the C ABI declared in include/ppcg.h.
//
// Method: Algorithm 2 (PIPECG) of Tiwari & Vadhiyar (Section III-B) with the
// Jacobi preconditioner (Section V-A), solving a sparse SPD system given in
// CSR.  See ppcg_kernels.hpp for the kernels of one iteration.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "ppcg_engine.hpp"
#include "ppcg_kernels.hpp"
#include "ppcg_pcg.hpp"
#include "ppcg_small.hpp"
#include "ppcg_setup.hpp"
#include "ppcg_fused.hpp"

namespace ppcg {

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

std::shared_mutex &release_mu()
{
    static std::shared_mutex m;
    return m;
}

void set_error(const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

static inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- arena
ppcg_status DevArena::alloc(size_t bytes)
{
    release();
    if (bytes == 0)
        bytes = 256;
    hipError_t e = hipMalloc((void **)&base, bytes);
    if (e != hipSuccess) {
        base = nullptr;
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PPCG_ERR_NOMEM : PPCG_ERR_DEVICE;
    }
    size = bytes;
    used = 0;
    return PPCG_OK;
}

void *DevArena::take(size_t bytes)
{
    const size_t a = (used + 255) & ~(size_t)255;
    if (a + bytes > size)
        return nullptr;
    used = a + bytes;
    return base + a;
}

void DevArena::release()
{
    if (base)
        (void)dev_free(base);
    base = nullptr;
    size = used = 0;
}

static size_t aligned(size_t b) { return (b + 255) & ~(size_t)255; }

// Check that [p, p + bytes) lies inside one device allocation of the current
// device, so that no kernel can fault on a wrong pointer or short buffer.
ppcg_status check_dev_range(const void *p, size_t bytes, const char *what)
{
    if (!p) {
        set_error("%s is NULL", what);
        return PPCG_ERR_INVALID_ARG;
    }
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        set_error("%s is not a device pointer", what);
        return PPCG_ERR_INVALID_ARG;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e == hipSuccess && base) {
        const char *b = (const char *)base, *q = (const char *)p;
        if (q + bytes > b + size) {
            set_error("%s: buffer of %zu bytes at offset %zu is shorter than the %zu bytes needed", what,
                      size, (size_t)(q - b), bytes);
            return PPCG_ERR_INVALID_ARG;
        }
    } else {
        (void)hipGetLastError();
    }
    return PPCG_OK;
}

// ---------------------------------------------------------------- byte model
// Algorithmic HBM bytes of one iteration.  PIPECG: the fused update reads 7
// vectors (n z w s p r dinv; u and q are scalings of r and s by the inverse
// diagonal, formed in registers) and writes 6 (z s p r w m), plus x read and
// written every other launch (two x-updates at once): 14 on average; the
// SpMV reads values and column indices of every
// stored entry, its row/chunk pointers, the input vector once, and writes one
// vector.  Classic PCG: the update reads x, p, r, s and the inverse diagonal
// and writes x, r, u (8 vectors); the SpMV reads u and the previous direction
// once each and writes the new direction and s (4 vectors) besides the matrix.
struct ByteModel {
    double vma, spmv;
};

static ByteModel byte_model(const ppcg_handle *h, int prec)
{
    const double ve = prec == PREC_F32 ? 4.0 : 8.0;   // vector element
    const bool pcg0 = h->opt.method == PPCG_METHOD_PCG || prec == PREC_F32;
    // matrix value: FP64, or a one-byte index into the value table (the
    // PIPECG SpMV with FP64 values), or FP32
    const double me = prec == PREC_F64 ? (h->vidx && !pcg0 ? 1.0 : 8.0) : 4.0;
    const double n = h->n;
    // FP32 vectors always iterate with Algorithm 1
    const bool pcg = h->opt.method == PPCG_METHOD_PCG || prec == PREC_F32;
    ByteModel bm;
    // a constant diagonal is read as one scalar: one vector stream fewer
    bm.vma = ((pcg ? 8.0 : 14.0) - (h->dinv_const ? 1.0 : 0.0)) * ve * n;
    const double ptr = h->fmt == FMT_SELL ? 8.0 * (h->nchunks + 1) : 4.0 * (n + 1);
    // the SpMVs read 16-bit column offsets when the matrix has them (not the
    // classic-PCG SpMV with FP32 values and FP64 vectors)
    // (none with the shared offset lists, which every iteration SpMV reads
    // when they are on: 4 bytes per chunk)
    const bool sh = h->shared_on;
    const double ie = sh ? 0.0 : (h->col16 && (PPCG_PCG_V32_COL16 || !(pcg && prec == PREC_V32))) ? 2.0 : 4.0;
    bm.spmv = (me + ie) * (double)h->nnz + ptr + (sh ? 4.0 * h->nchunks : 0.0) + (pcg ? 4.0 : 2.0) * ve * n;
    // the single-launch form keeps n in registers (neither written by the
    // SpMV nor read by the update) and, with a constant diagonal, forms
    // m = M^-1 w in the next launch's gathers instead of writing it (the
    // gathers read w in place of m)
    if (h->form == FORM_FUSED && prec == PREC_F64 && !pcg) {
        bm.vma -= (h->dinv_const ? 2.0 : 1.0) * ve * n;
        bm.spmv -= ve * n;
    }
    return bm;
}

// ---------------------------------------------------------------- SELL build
struct SellBuild {
    int sigma = 1;
    int nchunks = 0;
    int64_t stored = 0;
    int64_t *cptr = nullptr;
    int *col = nullptr;
    double *val = nullptr;
    int *perm = nullptr, *invperm = nullptr;
    int *cpat = nullptr, *pats = nullptr;  // shared offset lists (see k_sell_union)
    int npats = 0;
    void free_all()
    {
        if (cptr) (void)dev_free(cptr);
        if (col) (void)dev_free(col);
        if (val) (void)dev_free(val);
        if (perm) (void)dev_free(perm);
        if (invperm) (void)dev_free(invperm);
        if (cpat) (void)dev_free(cpat);
        if (pats) (void)dev_free(pats);
        *this = SellBuild();
    }
};

#define PPCG_HIP_CLEAN(call, cleanup)                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::ppcg::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),       \
                              __FILE__, __LINE__);                                         \
            cleanup;                                                                       \
            return e_ == hipErrorOutOfMemory ? PPCG_ERR_NOMEM : PPCG_ERR_DEVICE;           \
        }                                                                                  \
    } while (0)

// Chunk-size pass only: stored entries for a given sigma (for the autotuner).
static ppcg_status sell_size(hipStream_t s, int n, int sigma, const int *rowlen, int64_t *stored)
{
    const int nchunks = (n + kSellC - 1) / kSellC;
    int *perm = nullptr;
    int64_t *sz = nullptr, *cp = nullptr;
    auto clean = [&]() {
        if (perm) (void)dev_free(perm);
        if (sz) (void)dev_free(sz);
        if (cp) (void)dev_free(cp);
    };
    PPCG_HIP_CLEAN(hipMalloc(&sz, sizeof(int64_t) * nchunks), clean());
    PPCG_HIP_CLEAN(hipMalloc(&cp, sizeof(int64_t) * (nchunks + 1)), clean());
    if (sigma > 1) {
        PPCG_HIP_CLEAN(hipMalloc(&perm, sizeof(int) * n), clean());
        launch_sort_window(s, n, sigma, rowlen, perm);
    }
    k_chunk_size<<<blocks_for(nchunks, 256), 256, 0, s>>>(n, nchunks, perm, rowlen, sz);
    k_scan<<<1, 1024, 0, s>>>(nchunks, sz, cp);
    PPCG_HIP_CLEAN(hipMemcpyAsync(stored, cp + nchunks, sizeof(int64_t), hipMemcpyDeviceToHost, s), clean());
    PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
    clean();
    return PPCG_OK;
}

// Chunk widths for the shared offset lists of an unsorted SELL layout: sz
// holds 64 x each chunk's longest row (k_chunk_size); where a chunk's merged
// list is longer, its width grows to the list's length.  *ok is false (sz
// unchanged) when some chunk's list passes k_sell_union_count's cap or the
// widths grow by more than 1/32 in total: the lists would cost more padding
// than they save.
static ppcg_status widen_for_shared(hipStream_t s, int n, int nchunks, const int *rp, const int *ci, int64_t *sz,
                                    bool *ok)
{
    *ok = false;
    int *cnt = nullptr;
    PPCG_HIP(hipMalloc(&cnt, sizeof(int) * std::max(nchunks, 1)));
    std::vector<int> cnt_h((size_t)nchunks);
    std::vector<int64_t> sz_h((size_t)nchunks);
    k_sell_union_count<<<nchunks, kSellC, 0, s>>>(n, nchunks, rp, ci, sz, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(cnt_h.data(), cnt, sizeof(int) * nchunks, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sz_h.data(), sz, sizeof(int64_t) * nchunks, hipMemcpyDeviceToHost, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = es;
    (void)dev_free(cnt);
    PPCG_HIP(e);
    int64_t before = 0, after = 0;
    for (int c = 0; c < nchunks; ++c) {
        if (cnt_h[c] < 0)
            return PPCG_OK;
        const int64_t w = sz_h[c] / kSellC;
        before += w;
        after += std::max<int64_t>(w, cnt_h[c]);
        sz_h[c] = std::max<int64_t>(w, cnt_h[c]) * kSellC;
    }
    if (after * 32 > before * 33)
        return PPCG_OK;
    PPCG_HIP(hipMemcpyAsync(sz, sz_h.data(), sizeof(int64_t) * nchunks, hipMemcpyHostToDevice, s));
    PPCG_HIP(hipStreamSynchronize(s));
    *ok = true;
    return PPCG_OK;
}

// Shared offset lists of an unsorted SELL layout whose chunk extents sb.cptr
// are set (widened by widen_for_shared): each chunk's merged list
// (k_sell_union), the distinct lists concatenated on the host (a few KB for
// a stencil: one list per kind of boundary), and each chunk's list start.
// Leaves sb.cpat NULL when the distinct lists exceed kMaxSharedOffsets.
static ppcg_status build_shared_lists(hipStream_t s, int n, const int *rp, const int *ci, SellBuild &sb)
{
    const int64_t nl = sb.stored / kSellC;
    int *lists = nullptr;
    unsigned *flag = nullptr;
    auto clean = [&]() {
        if (lists) (void)dev_free(lists);
        if (flag) (void)dev_free(flag);
    };
    if (nl < 1 || sb.perm)
        return PPCG_OK;
    const unsigned zero = 0u;
    unsigned bad = 1u;
    PPCG_HIP_CLEAN(hipMalloc(&lists, sizeof(int) * nl), clean());
    PPCG_HIP_CLEAN(hipMalloc(&flag, sizeof(unsigned)), clean());
    PPCG_HIP_CLEAN(hipMemcpyAsync(flag, &zero, sizeof zero, hipMemcpyHostToDevice, s), clean());
    k_sell_union<<<sb.nchunks, kSellC, 0, s>>>(n, sb.nchunks, rp, ci, sb.cptr, lists, flag);
    PPCG_HIP_CLEAN(hipGetLastError(), clean());
    PPCG_HIP_CLEAN(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s), clean());
    PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
    if (bad) {
        clean();
        return PPCG_OK;
    }
    std::vector<int> lh((size_t)nl);
    std::vector<int64_t> cp((size_t)sb.nchunks + 1);
    PPCG_HIP_CLEAN(hipMemcpyAsync(lh.data(), lists, sizeof(int) * nl, hipMemcpyDeviceToHost, s), clean());
    PPCG_HIP_CLEAN(hipMemcpyAsync(cp.data(), sb.cptr, sizeof(int64_t) * cp.size(), hipMemcpyDeviceToHost, s),
                   clean());
    PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
    clean();
    lists = nullptr;
    flag = nullptr;
    std::map<std::string, int> seen;
    std::vector<int> pats, cpat((size_t)sb.nchunks);
    for (int c = 0; c < sb.nchunks; ++c) {
        const int64_t a = cp[c] / kSellC, len = (cp[c + 1] - cp[c]) / kSellC;
        std::string key((const char *)(lh.data() + a), (size_t)len * sizeof(int));
        auto it = seen.find(key);
        if (it == seen.end()) {
            if ((int64_t)pats.size() + len > kMaxSharedOffsets)
                return PPCG_OK;
            it = seen.emplace(std::move(key), (int)pats.size()).first;
            pats.insert(pats.end(), lh.begin() + a, lh.begin() + a + len);
        }
        cpat[c] = it->second;
    }
    if (pats.empty())
        pats.push_back(0);
    PPCG_HIP(hipMalloc(&sb.cpat, sizeof(int) * cpat.size()));
    PPCG_HIP(hipMalloc(&sb.pats, sizeof(int) * pats.size()));
    PPCG_HIP(hipMemcpyAsync(sb.cpat, cpat.data(), sizeof(int) * cpat.size(), hipMemcpyHostToDevice, s));
    PPCG_HIP(hipMemcpyAsync(sb.pats, pats.data(), sizeof(int) * pats.size(), hipMemcpyHostToDevice, s));
    PPCG_HIP(hipStreamSynchronize(s));
    sb.npats = (int)pats.size();
    return PPCG_OK;
}

// SELL-C-sigma storage of the CSR matrix.  shared: when the rows keep their
// order (sigma = 1) and every chunk has a shared offset list, the entries
// are placed on the lists (k_sell_fill_shared); the products of every row,
// and their order, stay those of its CSR entries.
static ppcg_status build_sell(hipStream_t s, int n, int sigma, const int *rp, const int *ci, const double *val,
                              const int *rowlen, SellBuild *out, bool shared)
{
    SellBuild sb;
    sb.sigma = sigma;
    sb.nchunks = (n + kSellC - 1) / kSellC;
    int64_t *sz = nullptr;
    auto clean = [&]() {
        if (sz) (void)dev_free(sz);
        sb.free_all();
    };
    PPCG_HIP_CLEAN(hipMalloc(&sz, sizeof(int64_t) * sb.nchunks), clean());
    PPCG_HIP_CLEAN(hipMalloc(&sb.cptr, sizeof(int64_t) * (sb.nchunks + 1)), clean());
    if (sigma > 1) {
        PPCG_HIP_CLEAN(hipMalloc(&sb.perm, sizeof(int) * n), clean());
        PPCG_HIP_CLEAN(hipMalloc(&sb.invperm, sizeof(int) * n), clean());
        launch_sort_window(s, n, sigma, rowlen, sb.perm);
        k_invert_perm<<<blocks_for(n, 256), 256, 0, s>>>(n, sb.perm, sb.invperm);
    }
    k_chunk_size<<<blocks_for(sb.nchunks, 256), 256, 0, s>>>(n, sb.nchunks, sb.perm, rowlen, sz);
    bool widened = false;
    if (shared && sigma == 1) {
        const ppcg_status rc = widen_for_shared(s, n, sb.nchunks, rp, ci, sz, &widened);
        if (rc < 0) {
            clean();
            return rc;
        }
    }
    k_scan<<<1, 1024, 0, s>>>(sb.nchunks, sz, sb.cptr);
    PPCG_HIP_CLEAN(hipMemcpyAsync(&sb.stored, sb.cptr + sb.nchunks, sizeof(int64_t), hipMemcpyDeviceToHost, s),
                   clean());
    PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
    PPCG_HIP_CLEAN(hipMalloc(&sb.col, sizeof(int) * std::max<int64_t>(sb.stored, 1)), clean());
    PPCG_HIP_CLEAN(hipMalloc(&sb.val, sizeof(double) * std::max<int64_t>(sb.stored, 1)), clean());
    if (widened) {
        const ppcg_status rc = build_shared_lists(s, n, rp, ci, sb);
        if (rc < 0) {
            clean();
            return rc;
        }
    }
    if (sb.cpat) {
        unsigned *flag = nullptr;
        const unsigned zero = 0u;
        unsigned bad = 1u;
        hipError_t e = hipMalloc(&flag, sizeof(unsigned));
        if (e == hipSuccess)
            e = hipMemcpyAsync(flag, &zero, sizeof zero, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            k_sell_fill_shared<<<blocks_for((size_t)sb.nchunks * kSellC, 256), 256, 0, s>>>(
                n, sb.nchunks, rp, ci, val, sb.cptr, sb.cpat, sb.pats, sb.col, sb.val, flag);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s);
        const hipError_t es = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = es;
        if (flag)
            (void)dev_free(flag);
        PPCG_HIP_CLEAN(e, clean());
        if (bad) {
            set_error("shared offset lists: an entry found no place");
            clean();
            return PPCG_ERR_DEVICE;
        }
    } else {
        k_sell_fill<<<blocks_for((size_t)sb.nchunks * kSellC, 256), 256, 0, s>>>(
            n, sb.nchunks, rp, ci, val, sb.perm, sb.invperm, sb.cptr, sb.col, sb.val);
        PPCG_HIP_CLEAN(hipGetLastError(), clean());
    }
    (void)dev_free(sz);
    sz = nullptr;
    *out = sb;
    return PPCG_OK;
}

// ---------------------------------------------------------------- autotuner
// Candidate SpMV configurations are timed on the matrix itself: five timed
// SpMV executions each (after one warm-up), the same count the paper's
// performance model uses to measure SpMV speed (Section IV-C).  Choices are
// cached per coarse matrix signature.
struct TuneKey {
    int logn, mean, cv10, maxlen_log;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(logn, mean, cv10, maxlen_log) < std::tie(o.logn, o.mean, o.cv10, o.maxlen_log);
    }
};
struct TuneVal {
    int fmt, sigma, lanes;
    int col16;  // SELL: 1 when the 16-bit column offsets timed faster
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune_cache;
// Signatures being tuned: one thread tunes a signature at a time, and
// the others wait for its choice, so every handle of a signature gets the
// same layout (the layout decides the summation order of the results).
static std::set<TuneKey> g_tuning;
static std::condition_variable g_tune_cv;

ppcg_status fill_desc(ppcg_handle *h, int prec, SysState *st, SysDesc *d, double tol, int fixed, int maxit,
                      int stop, int vals32)
{
    PrecData &pd = prec == PREC_F64 ? h->f64 : h->f32;
    if (!pd.ready) {
        set_error("precision data not prepared");
        return PPCG_ERR_INVALID_ARG;
    }
    memset(d, 0, sizeof *d);
    d->n = h->n;
    d->ntiles = h->ntiles;
    d->fmt = h->fmt;
    d->lanes = h->lanes;
    d->stop = stop;
    d->maxit = maxit;
    d->fixed = fixed;
    d->prec = prec;
    d->pair = -1;
    d->tol = tol;
    d->cptr = h->cptr;
    d->rp = h->rp;
    d->col = h->col;
    d->col16 = h->col16;
    d->vidx = h->vidx;
    d->vtab = h->vtab;
    d->nvtab = h->nvtab;
    d->cpat = h->shared_on ? h->cpat : nullptr;
    d->pats = h->pats;
    d->val = pd.val;
    d->val32 = h->val32;
    d->vals32 = vals32;
    if (vals32 && !h->val32) {
        set_error("FP32 values not prepared");
        return PPCG_ERR_INVALID_ARG;
    }
    d->dinv = pd.dinv;
    d->dinv_const = h->dinv_const ? 1 : 0;
    d->x = pd.vec[VX];
    d->r = pd.vec[VR];
    d->u = pd.vec[VU];
    d->w = pd.vec[VW];
    d->m = pd.vec[VM];
    d->nv = pd.vec[VN];
    d->z = pd.vec[VZ];
    d->q = pd.vec[VQ];
    d->s = pd.vec[VS];
    d->p = pd.vec[VP];
    d->b = pd.vec[VB];
    d->part = prec == PREC_F64 ? h->part : h->part32;
    d->st = st;
    d->frows = fused_tile_rows(h->n, h->cus);
    d->nftiles = (h->n + d->frows - 1) / d->frows;
    d->frec = h->frec;
    d->fpart = h->fpart;
    d->w1 = h->w1;
    return PPCG_OK;
}

int fused_tiles(const ppcg_handle *h)
{
    const int fr = fused_tile_rows(h->n, h->cus);
    return (h->n + fr - 1) / fr;
}

ppcg_status ensure_fused(ppcg_handle *h)
{
    if (h->frec)
        return PPCG_OK;
    const size_t nft = (size_t)fused_tiles(h);
    const size_t pb = 2 * nft * 4 * sizeof(double), vb = (size_t)h->n * sizeof(double);
    PPCG_TRY(h->fused_arena.alloc(2 * sizeof(SysState) + pb + vb + 3 * 256));
    h->frec = (SysState *)h->fused_arena.take(2 * sizeof(SysState));
    h->fpart = (double *)h->fused_arena.take(pb);
    h->w1 = (double *)h->fused_arena.take(vb);
    return PPCG_OK;
}

// Upload a single-system descriptor (all tiles) for direct kernel launches.
static ppcg_status plain_setup(ppcg_handle *h, double tol, int fixed, int maxit)
{
    hipStream_t s = h->stream;
    if (!h->plain_desc) {
        PPCG_HIP(hipMalloc(&h->plain_desc, sizeof(SysDesc)));
        PPCG_HIP(hipMalloc(&h->plain_st, sizeof(SysState)));
        PPCG_HIP(hipMalloc(&h->plain_tab, sizeof(WorkItem) * h->ntiles));
        PPCG_HIP(hipMalloc(&h->plain_cnt, sizeof(int) * 2));  // [1]: fused tiles
        std::vector<WorkItem> th(h->ntiles);
        for (int t = 0; t < h->ntiles; ++t)
            th[t] = {0, t};
        const int count[2] = {h->ntiles, fused_tiles(h)};
        PPCG_HIP(hipMemcpyAsync(h->plain_tab, th.data(), sizeof(WorkItem) * count[0], hipMemcpyHostToDevice, s));
        PPCG_HIP(hipMemcpyAsync(h->plain_cnt, count, sizeof count, hipMemcpyHostToDevice, s));
        PPCG_HIP(hipStreamSynchronize(s));  // host sources are about to go out of scope
    }
    SysDesc dh;
    PPCG_TRY(fill_desc(h, PREC_F64, h->plain_st, &dh, tol, fixed, maxit, STOP_REL));
    PPCG_HIP(hipMemcpyAsync(h->plain_desc, &dh, sizeof dh, hipMemcpyHostToDevice, s));
    PPCG_HIP(hipMemsetAsync(h->plain_st, 0, sizeof(SysState), s));
    PPCG_HIP(hipStreamSynchronize(s));
    return PPCG_OK;
}

static void plain_free(ppcg_handle *h)
{
    if (h->plain_desc) (void)dev_free(h->plain_desc);
    if (h->plain_st) (void)dev_free(h->plain_st);
    if (h->plain_tab) (void)dev_free(h->plain_tab);
    if (h->plain_cnt) (void)dev_free(h->plain_cnt);
    h->plain_desc = nullptr;
    h->plain_st = nullptr;
    h->plain_tab = nullptr;
    h->plain_cnt = nullptr;
}

// Time `reps` SpMV launches of the handle's current format (MODE_PLAIN).
static ppcg_status time_spmv(ppcg_handle *h, int reps, double *ms)
{
    hipStream_t s = h->stream;
    PPCG_TRY(plain_setup(h, 1e-8, 0, 1));
    k_fill<double><<<blocks_for(h->n, 256), 256, 0, s>>>((size_t)h->n, (double *)h->f64.vec[VX], 1.0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto clean = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    PPCG_HIP_CLEAN(hipEventCreate(&e0), clean());
    PPCG_HIP_CLEAN(hipEventCreate(&e1), clean());
    k_spmv<double, MODE_PLAIN><<<h->ntiles, kSpmvThreads, 0, s>>>(h->plain_tab, h->plain_cnt, h->plain_desc, PPCG_XCD_REMAP_SPMV);
    PPCG_HIP_CLEAN(hipEventRecord(e0, s), clean());
    for (int i = 0; i < reps; ++i)
        k_spmv<double, MODE_PLAIN><<<h->ntiles, kSpmvThreads, 0, s>>>(h->plain_tab, h->plain_cnt, h->plain_desc,
                                                                      PPCG_XCD_REMAP_SPMV);
    PPCG_HIP_CLEAN(hipEventRecord(e1, s), clean());
    PPCG_HIP_CLEAN(hipEventSynchronize(e1), clean());
    float f = 0.f;
    PPCG_HIP_CLEAN(hipEventElapsedTime(&f, e0, e1), clean());
    *ms = f / reps;
    clean();
    return PPCG_OK;
}

static void free_matrix(ppcg_handle *h)
{
    if (h->cptr) (void)dev_free(h->cptr);
    if (h->rp) (void)dev_free(h->rp);
    if (h->col) (void)dev_free(h->col);
    if (h->col16) (void)dev_free(h->col16);
    h->col16 = nullptr;
    if (h->vidx) (void)dev_free(h->vidx);
    if (h->vtab) (void)dev_free(h->vtab);
    h->vidx = nullptr;
    h->vtab = nullptr;
    h->nvtab = 0;
    if (h->val64) (void)dev_free(h->val64);
    if (h->val32) (void)dev_free(h->val32);
    if (h->perm) (void)dev_free(h->perm);
    if (h->invperm) (void)dev_free(h->invperm);
    if (h->cpat) (void)dev_free(h->cpat);
    if (h->pats) (void)dev_free(h->pats);
    h->cpat = h->pats = nullptr;
    h->npats = 0;
    h->shared_on = false;
    h->cptr = nullptr;
    h->rp = h->col = h->perm = h->invperm = nullptr;
    h->val64 = nullptr;
    h->val32 = nullptr;
}

static ppcg_status adopt_sell(ppcg_handle *h, SellBuild &sb)
{
    free_matrix(h);
    h->fmt = FMT_SELL;
    h->sigma = sb.sigma;
    h->lanes = 0;
    h->nchunks = sb.nchunks;
    h->nnz_stored = sb.stored;
    h->cptr = sb.cptr;
    h->col = sb.col;
    h->val64 = sb.val;
    h->perm = sb.perm;
    h->invperm = sb.invperm;
    h->cpat = sb.cpat;
    h->pats = sb.pats;
    h->npats = sb.npats;
    sb = SellBuild();
    return PPCG_OK;
}

// 16-bit column offsets from the row, when every one fits (banded matrices,
// stencils whose plane has at most 32767 points): half the index bytes.
// Sets *built; a matrix whose offsets do not fit keeps its 32-bit columns.
static ppcg_status build_col16(ppcg_handle *h, bool *built)
{
    *built = false;
    short *c16 = nullptr;
    unsigned *flag = nullptr;
    unsigned nofit = 1u;
    const unsigned zero = 0u;
    hipStream_t s = h->stream;
    PPCG_HIP(hipMalloc(&c16, sizeof(short) * std::max<int64_t>(h->nnz_stored, 1)));
    hipError_t e = hipMalloc(&flag, sizeof(unsigned));
    if (e == hipSuccess)
        e = hipMemcpyAsync(flag, &zero, sizeof zero, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_sell_delta16<<<blocks_for((size_t)h->nchunks * kSellC, 256), 256, 0, s>>>(h->nchunks, h->cptr, h->col,
                                                                                    c16, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nofit, flag, sizeof nofit, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (flag)
        (void)dev_free(flag);
    if (e != hipSuccess || nofit) {
        (void)dev_free(c16);
        c16 = nullptr;
    }
    PPCG_HIP(e);
    h->col16 = c16;
    *built = c16 != nullptr;
    return PPCG_OK;
}

static void drop_col16(ppcg_handle *h)
{
    if (h->col16)
        (void)dev_free(h->col16);
    h->col16 = nullptr;
}

static ppcg_status time_spmv(ppcg_handle *h, int reps, double *ms);

// SELL: whether the SpMVs read 16-bit column offsets.  They halve the index
// bytes but cost an unpack per entry pair and a sub-dword load for an odd
// tail; on gfx950 that wins for long rows (27-point stencils) and loses for
// short ones (7-point), so both are timed on the matrix and the faster is
// kept.  The two layouts are timed twice in alternation (five SpMVs each
// time, after a warm-up) and the best of each pair compared; 16-bit offsets
// must win by 2 %, so that timing noise cannot pick them for a matrix where
// they are slower.  `known` >= 0 replays a cached decision;
// PPCG_FLAG_SELL_COL16 / _COL32 force the choice.  Off entirely when
// PPCG_SELL_COL16 is 0.
static ppcg_status tune_col16(ppcg_handle *h, int known, int *chosen)
{
    *chosen = 0;
    if (h->opt.flags & PPCG_FLAG_SELL_COL16)
        known = 1;
    else if (h->opt.flags & PPCG_FLAG_SELL_COL32)
        known = 0;
    if (!PPCG_SELL_COL16 || h->fmt != FMT_SELL || known == 0)
        return PPCG_OK;
    bool built = false;
    PPCG_TRY(build_col16(h, &built));
    if (!built)
        return PPCG_OK;
    if (known < 0) {
        short *c16 = h->col16;
        double t32 = 1e300, t16 = 1e300;
        for (int round = 0; round < 2; ++round) {
            double t = 0.0;
            h->col16 = nullptr;  // the SpMV reads the 32-bit columns
            ppcg_status rc = time_spmv(h, 5, &t);
            h->col16 = c16;
            PPCG_TRY(rc);
            t32 = std::min(t32, t);
            PPCG_TRY(time_spmv(h, 5, &t));
            t16 = std::min(t16, t);
        }
        if (!(t16 < 0.98 * t32)) {
            drop_col16(h);
            return PPCG_OK;
        }
    }
    *chosen = 1;
    return PPCG_OK;
}

// A set of at most kMaxValueTable 64-bit keys (open addressing, load at
// most 1/4); add() fails when a new key would exceed that count.
struct ValueSet {
    static constexpr int kSlots = 4 * kMaxValueTable;
    uint64_t slot[kSlots];
    bool used[kSlots] = {};
    int count = 0;
    uint64_t last = 0;
    bool have_last = false;
    bool add(uint64_t k)
    {
        if (have_last && k == last)  // runs of equal values are common
            return true;
        last = k;
        have_last = true;
        unsigned p = (unsigned)((k * 0x9E3779B97F4A7C15ull) >> 54);  // 10 bits
        while (used[p]) {
            if (slot[p] == k)
                return true;
            p = (p + 1) & (kSlots - 1);
        }
        if (count == kMaxValueTable)
            return false;
        used[p] = true;
        slot[p] = k;
        ++count;
        return true;
    }
    // false as soon as a value does not fit (or *stop is raised)
    bool scan(const double *v, int64_t m, const std::atomic<bool> *stop = nullptr)
    {
        for (int64_t i = 0; i < m; ++i) {
            if (stop && (i & 0xffff) == 0 && stop->load(std::memory_order_relaxed))
                return false;
            uint64_t k;
            memcpy(&k, v + i, sizeof k);
            if (!add(k))
                return false;
        }
        return true;
    }
};

// The matrix's distinct values as ascending bit patterns, +0.0 (the SELL
// padding) included, when there are at most kMaxValueTable of them (*fits).
// A scan stops at the first value past that count, so a matrix with many
// values costs little.  Host CSR values are scanned by up to 8 threads, each
// over its own range, and their sets merged; device values are copied in
// chunks and scanned in turn.
static ppcg_status distinct_values(const ppcg_handle *h, const double *val_host, const double *val_dev,
                                   std::vector<uint64_t> *keys, bool *fits)
{
    *fits = false;
    auto merged = std::make_unique<ValueSet>();
    if (!merged->add(0))  // +0.0
        return PPCG_OK;
    if (val_host) {
        const int64_t nnz = h->nnz;
        const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(8, nnz / (1 << 20)));
        std::vector<std::unique_ptr<ValueSet>> sets;
        for (int t = 0; t < nt; ++t)
            sets.push_back(std::make_unique<ValueSet>());
        std::vector<char> ok(nt, 1);
        std::atomic<bool> stop(false);
        auto work = [&](int t) {
            const int64_t lo = nnz * t / nt, hi = nnz * (t + 1) / nt;
            ok[t] = sets[t]->scan(val_host + lo, hi - lo, &stop);
            if (!ok[t])
                stop.store(true);
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t)
            th.emplace_back(work, t);
        work(0);
        for (auto &x : th)
            x.join();
        for (int t = 0; t < nt; ++t) {
            if (!ok[t])
                return PPCG_OK;
            for (int p = 0; p < ValueSet::kSlots; ++p)
                if (sets[t]->used[p] && !merged->add(sets[t]->slot[p]))
                    return PPCG_OK;
        }
    } else {
        constexpr int64_t kChunk = 1 << 20;
        std::vector<double> buf((size_t)std::min<int64_t>(h->nnz, kChunk));
        for (int64_t off = 0; off < h->nnz; off += kChunk) {
            const int64_t m = std::min(kChunk, h->nnz - off);
            PPCG_HIP(hipMemcpyAsync(buf.data(), val_dev + off, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
            PPCG_HIP(hipStreamSynchronize(h->stream));
            if (!merged->scan(buf.data(), m))
                return PPCG_OK;
        }
    }
    keys->clear();
    for (int p = 0; p < ValueSet::kSlots; ++p)
        if (merged->used[p])
            keys->push_back(merged->slot[p]);
    std::sort(keys->begin(), keys->end());
    *fits = true;
    return PPCG_OK;
}

// Build the one-byte value indices of the stored SELL values and the table.
static ppcg_status build_vtab(ppcg_handle *h, const std::vector<uint64_t> &keys)
{
    hipStream_t s = h->stream;
    const int nt = (int)keys.size();
    unsigned char *vi = nullptr;
    double *tab = nullptr;
    unsigned *flag = nullptr;
    unsigned zero = 0u, bad = 0u;
    hipError_t e = hipMalloc(&vi, (size_t)std::max<int64_t>(h->nnz_stored, 1));
    if (e == hipSuccess)
        e = hipMalloc(&tab, sizeof(double) * nt);
    if (e == hipSuccess)
        e = hipMalloc(&flag, sizeof(unsigned));
    if (e == hipSuccess)
        e = hipMemcpyAsync(tab, keys.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(flag, &zero, sizeof zero, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && h->nnz_stored > 0) {
        k_sell_vidx<<<blocks_for((size_t)h->nnz_stored, 256), 256, 0, s>>>(
            h->nnz_stored, h->val64, (const unsigned long long *)tab, nt, vi, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s);
    // always: the copies above read and write host memory of this frame
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = es;
    if (flag)
        (void)dev_free(flag);
    if (e != hipSuccess || bad) {
        if (vi) (void)dev_free(vi);
        if (tab) (void)dev_free(tab);
        vi = nullptr;
        tab = nullptr;
    }
    PPCG_HIP(e);
    h->vidx = vi;
    h->vtab = tab;
    h->nvtab = vi ? nt : 0;
    return PPCG_OK;
}

static void drop_vtab(ppcg_handle *h)
{
    if (h->vidx) (void)dev_free(h->vidx);
    if (h->vtab) (void)dev_free(h->vtab);
    h->vidx = nullptr;
    h->vtab = nullptr;
    h->nvtab = 0;
}

// SELL: whether the FP64 SpMVs read a one-byte index per stored entry into a
// table of the matrix's distinct values instead of the 8-byte value, when
// there are at most 256 of them (index-and-value compression, as in CSR-VI:
// Kourtis, Goumas and Koziris, 2008).  Exact: the table holds the values
// themselves, so the products are the same.  Constant-coefficient stencils
// have two or three values; most assembled matrices have too many, and the
// scan gives up early.  Both layouts are timed like the column layouts
// (alternated), and the table is kept unless it made the SpMV more than 2 %
// slower: the timed two-launch SpMV of a short-row system is bound by
// latency and shows the saved bytes little (7-point rows: 2-3 %), while the
// single-launch iteration, where most such systems end up, gains from them
// (7-point 128^3: with the 16-bit columns 66.7 -> 56.6 us per iteration;
// a batch of 256 2-D systems kept the table for 109 of them under a rule of
// a 5 % gain per iteration).  The 125-point rows' SpMV ran 1.45x faster.
// The decision is cached per (rows, mean row length) signature: a
// matrix of a signature whose table lost is not scanned, one whose table
// won keeps its table when it has one, untimed.  PPCG_FLAG_SELL_VALUE_TABLE /
// _FULL_VALUES force the choice, and PPCG_SELL_VTAB = 0 switches it off.
// Timed value-table decisions by (log2 of the row count, mean stored row
// length): a signature whose table lost is not scanned again.
static std::map<std::pair<int, int>, bool> g_vtab_kept;

static ppcg_status tune_vtab(ppcg_handle *h, const double *val_host, const double *val_dev)
{
    const unsigned fl = h->opt.flags;
    if (!PPCG_SELL_VTAB || h->fmt != FMT_SELL || (fl & PPCG_FLAG_SELL_FULL_VALUES))
        return PPCG_OK;
    const std::pair<int, int> sig((int)std::log2((double)h->n), (int)std::lround((double)h->nnz_stored / h->n));
    bool known = false, kept = false;
    if (!(fl & PPCG_FLAG_SELL_VALUE_TABLE)) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_vtab_kept.find(sig);
        if (it != g_vtab_kept.end()) {
            known = true;
            kept = it->second;
        }
    }
    // (a system the one-workgroup kernel iterates always takes the table)
    if (known && !kept && h->n > PPCG_SMALL_MAX_ROWS)
        return PPCG_OK;
    std::vector<uint64_t> keys;
    bool fits = false;
    PPCG_TRY(distinct_values(h, val_host, val_dev, &keys, &fits));
    if (!fits)
        return PPCG_OK;
    PPCG_TRY(build_vtab(h, keys));
    if (!h->vidx || (fl & PPCG_FLAG_SELL_VALUE_TABLE) || known)
        return PPCG_OK;
    unsigned char *vi = h->vidx;
    double tf = 1e300, tv = 1e300;
    for (int round = 0; round < 2; ++round) {
        double t = 0.0;
        h->vidx = nullptr;  // the SpMV reads the values
        ppcg_status rc = time_spmv(h, 5, &t);
        h->vidx = vi;
        PPCG_TRY(rc);
        tf = std::min(tf, t);
        PPCG_TRY(time_spmv(h, 5, &t));
        tv = std::min(tv, t);
    }
    // systems the one-workgroup kernel iterates keep the table: it stages the
    // matrix in LDS through it
    const bool keep = tv <= 1.02 * tf || h->n <= PPCG_SMALL_MAX_ROWS;
    if (!keep)
        drop_vtab(h);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_vtab_kept[sig] = keep;
    return PPCG_OK;
}

// SELL on shared offset lists: whether the FP64 PIPECG SpMV reads each
// chunk's list (through the scalar cache) instead of a column per entry.
// It saves the column bytes (2 or 4 per entry) and the wait of every gather
// on its column load, and costs a clamp per entry.  Timed like the value
// table (alternated, best of two) and kept when 2 % faster; decisions are
// cached per (rows, mean stored row length, value table, 16-bit columns)
// signature.  PPCG_FLAG_SELL_SHARED_OFFSETS / _NO_SHARED_OFFSETS force it;
// a forced column layout (PPCG_FLAG_SELL_COL16 / _COL32) leaves it off.
static std::map<std::tuple<int, int, int, int>, bool> g_shared_kept;

static ppcg_status tune_shared(ppcg_handle *h)
{
    h->shared_on = false;
    const unsigned fl = h->opt.flags;
    if (!h->cpat || h->fmt != FMT_SELL || (fl & PPCG_FLAG_SELL_NO_SHARED_OFFSETS))
        return PPCG_OK;
    if (fl & PPCG_FLAG_SELL_SHARED_OFFSETS) {
        h->shared_on = true;
        return PPCG_OK;
    }
    if (fl & (PPCG_FLAG_SELL_COL16 | PPCG_FLAG_SELL_COL32))  // a column layout was pinned
        return PPCG_OK;
    const auto sig = std::make_tuple((int)std::log2((double)h->n), (int)std::lround((double)h->nnz_stored / h->n),
                                     h->vidx ? 1 : 0, h->col16 ? 1 : 0);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_shared_kept.find(sig);
        if (it != g_shared_kept.end()) {
            h->shared_on = it->second;
            return PPCG_OK;
        }
    }
    double tc = 1e300, ts = 1e300;
    for (int round = 0; round < 2; ++round) {
        double t = 0.0;
        h->shared_on = false;
        PPCG_TRY(time_spmv(h, 5, &t));
        tc = std::min(tc, t);
        h->shared_on = true;
        PPCG_TRY(time_spmv(h, 5, &t));
        ts = std::min(ts, t);
    }
    h->shared_on = ts < 0.98 * tc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_shared_kept[sig] = h->shared_on;
    return PPCG_OK;
}

// The single-launch form reads the shared lists whenever the matrix has them
// (unless a column layout is pinned or the lists are refused): there the
// SpMV's column loads sit in the chain of every row, and the lists measured
// within 1 % or faster on every stencil tried, also where the two-launch
// SpMV alone is a few percent slower with them (µs per iteration, per-entry
// columns against lists: 7-point 128^3 51.0 / 50.5, 27-point 160^3
// 298 / 260, 125-point 100^3 142 / 118, 5-point 2048^2 90.3 / 91.2; the 256
// 2-D systems of a batch 67.8 / 65.0 ms).
static void shared_for_fused(ppcg_handle *h)
{
    const unsigned fl = h->opt.flags;
    if (h->form == FORM_FUSED && h->cpat && !h->shared_on &&
        !(fl & (PPCG_FLAG_SELL_NO_SHARED_OFFSETS | PPCG_FLAG_SELL_COL16 | PPCG_FLAG_SELL_COL32)))
        h->shared_on = true;
}

// ---------------------------------------------------------------- iteration form
// Time kIters iterations of each form of FP64 PIPECG on the handle's stored
// matrix, after their initialisations, from b = 1 and x0 = 0 in fixed-
// iteration mode.  *ms_two and *ms_fused: milliseconds per iteration (launch
// gaps included, kernels launched directly); *valid is false when a
// sequence stopped early (the timing would not be an iteration's).
static ppcg_status time_forms(ppcg_handle *h, double *ms_two, double *ms_fused, bool *valid)
{
    constexpr int kIters = 16;
    hipStream_t s = h->stream;
    PPCG_TRY(plain_setup(h, 0.0, INT_MAX, INT_MAX));
    const int n = h->n, grid = h->ntiles, fgrid = fused_tiles(h);
    const WorkItem *tab = h->plain_tab;
    const int *cnt = h->plain_cnt;
    const SysDesc *dd = h->plain_desc;
    hipEvent_t ev[4] = {};
    auto clean = [&]() {
        (void)hipStreamSynchronize(s);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto &e : ev)
        PPCG_HIP_CLEAN(hipEventCreate(&e), clean());
    *valid = true;
    float best[2] = {1e30f, 1e30f};
    for (int round = 0; round < 2; ++round) {
        for (int form = 0; form < 2; ++form) {
            k_fill<double><<<blocks_for(n, 256), 256, 0, s>>>((size_t)n, (double *)h->f64.vec[VB], 1.0);
            k_fill<double><<<blocks_for(n, 256), 256, 0, s>>>((size_t)n, (double *)h->f64.vec[VX], 0.0);
            if (form == 0) {
                launch_pipecg_init(s, tab, cnt, dd, grid);
                PPCG_HIP_CLEAN(hipEventRecord(ev[0], s), clean());
                for (int i = 0; i < kIters; ++i)
                    launch_pipecg_iter(s, tab, cnt, dd, grid, PPCG_XCD_REMAP);
                PPCG_HIP_CLEAN(hipEventRecord(ev[1], s), clean());
            } else {
                launch_pipecg_init_fused(s, tab, cnt, dd, grid);
                k_fused_begin<<<fgrid, 64, 0, s>>>(tab, cnt + 1, dd);
                // the first launch ends the initialisation (no update)
                k_fused<<<fgrid, kFusedThreads, 0, s>>>(tab, cnt + 1, dd, PPCG_FUSED_REMAP, 0);
                PPCG_HIP_CLEAN(hipEventRecord(ev[2], s), clean());
                for (int i = 1; i <= kIters; ++i)
                    k_fused<<<fgrid, kFusedThreads, 0, s>>>(tab, cnt + 1, dd, PPCG_FUSED_REMAP, i & 1);
                PPCG_HIP_CLEAN(hipEventRecord(ev[3], s), clean());
            }
            PPCG_HIP_CLEAN(hipGetLastError(), clean());
            SysState st;
            PPCG_HIP_CLEAN(hipMemcpyAsync(&st, h->plain_st, sizeof st, hipMemcpyDeviceToHost, s), clean());
            PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
            if (st.done)
                *valid = false;
            float ms = 0.f;
            PPCG_HIP_CLEAN(hipEventElapsedTime(&ms, ev[2 * form], ev[2 * form + 1]), clean());
            best[form] = std::min(best[form], ms);
        }
    }
    *ms_two = best[0] / kIters;
    *ms_fused = best[1] / kIters;
    clean();
    return PPCG_OK;
}

// Decisions per (rows on a log scale, stored entries per row, 16-bit columns,
// value table, sorted rows): 1 = single-launch form.  One thread times a
// signature at a time, so concurrent creates get the same form (and the same
// arithmetic).
static std::map<std::tuple<int, int, int, int, int>, int> g_form_cache;
static std::set<std::tuple<int, int, int, int, int>> g_form_tuning;

static void drop_fused(ppcg_handle *h)
{
    h->fused_arena.release();
    h->frec = nullptr;
    h->fpart = nullptr;
    h->w1 = nullptr;
}

// Choose the iteration form of FP64 PIPECG for the stored matrix (SELL only):
// forced by PPCG_FLAG_ITER_FUSED / PPCG_FLAG_ITER_TWO_LAUNCH, else the two
// launches for systems the one-workgroup kernel takes, else the faster of
// the two forms timed on this matrix.
static ppcg_status tune_form(ppcg_handle *h)
{
    h->form = FORM_TWO;
    const uint32_t f = h->opt.flags;
    if ((f & PPCG_FLAG_ITER_TWO_LAUNCH) || h->fmt != FMT_SELL)
        return PPCG_OK;
    if (f & PPCG_FLAG_ITER_FUSED) {
        PPCG_TRY(ensure_fused(h));
        h->form = FORM_FUSED;
        return PPCG_OK;
    }
    if (h->n <= PPCG_SMALL_MAX_ROWS)
        return PPCG_OK;
    const auto key = std::make_tuple((int)std::log2((double)h->n),
                                     (int)std::lround((double)h->nnz_stored / h->n), h->col16 ? 1 : 0,
                                     h->vidx ? 1 : 0, h->sigma > 1 ? 1 : h->shared_on ? 2 : 0);
    {
        std::unique_lock<std::mutex> lk(g_tune_mu);
        g_tune_cv.wait(lk, [&] { return !g_form_tuning.count(key); });
        auto it = g_form_cache.find(key);
        if (it != g_form_cache.end()) {
            lk.unlock();
            if (it->second == FORM_FUSED) {
                PPCG_TRY(ensure_fused(h));
                h->form = FORM_FUSED;
            }
            return PPCG_OK;
        }
        g_form_tuning.insert(key);
    }
    struct Release {
        std::tuple<int, int, int, int, int> k;
        ~Release()
        {
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_form_tuning.erase(k);
            }
            g_tune_cv.notify_all();
        }
    } release{key};
    PPCG_TRY(ensure_fused(h));
    double t2 = 0, tf = 0;
    bool valid = false;
    PPCG_TRY(time_forms(h, &t2, &tf, &valid));
    const int form = valid && tf < t2 ? FORM_FUSED : FORM_TWO;
    if (form == FORM_FUSED)
        h->form = FORM_FUSED;
    else
        drop_fused(h);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (valid)
        g_form_cache[key] = form;
    return PPCG_OK;
}

static ppcg_status adopt_csrv(ppcg_handle *h, int lanes, const int *rp, const int *ci, const double *val)
{
    free_matrix(h);
    h->fmt = FMT_CSRV;
    h->sigma = 1;
    h->lanes = lanes;
    h->nchunks = 0;
    h->nnz_stored = h->nnz;
    PPCG_HIP(hipMalloc(&h->rp, sizeof(int) * (h->n + 1)));
    PPCG_HIP(hipMalloc(&h->col, sizeof(int) * std::max<int64_t>(h->nnz, 1)));
    PPCG_HIP(hipMalloc(&h->val64, sizeof(double) * std::max<int64_t>(h->nnz, 1)));
    PPCG_HIP(hipMemcpyAsync(h->rp, rp, sizeof(int) * (h->n + 1), hipMemcpyDeviceToDevice, h->stream));
    PPCG_HIP(hipMemcpyAsync(h->col, ci, sizeof(int) * h->nnz, hipMemcpyDeviceToDevice, h->stream));
    PPCG_HIP(hipMemcpyAsync(h->val64, val, sizeof(double) * h->nnz, hipMemcpyDeviceToDevice, h->stream));
    return PPCG_OK;
}

// Point the FP64 precision data at the current matrix storage (dinv in
// stored-row order).
static ppcg_status bind_f64(ppcg_handle *h, const double *dinv_orig)
{
    PrecData &pd = h->f64;
    pd.prec = PREC_F64;
    pd.val = h->val64;
    k_permute_d<<<blocks_for(h->n, 256), 256, 0, h->stream>>>(h->n, h->perm, dinv_orig, h->dinv64);
    PPCG_HIP(hipGetLastError());
    pd.dinv = h->dinv64;
    pd.ready = true;
    return PPCG_OK;
}

// Lanes per row of the CSR-vector format when it is forced (no timing): the
// power of two in [2, 64] nearest above half the mean row length.
int csrv_default_lanes(double mean)
{
    int l = 2;
    while (l < 64 && l < mean / 2)
        l <<= 1;
    return l;
}

static ppcg_status choose_format(ppcg_handle *h, const int *rp, const int *ci, const double *val, const int *rowlen,
                                 const double *dinv_orig, const std::vector<int> &rowlen_h)
{
    const ppcg_spmv_format want = h->opt.spmv_format;
    // a forced 16-bit column choice is not a timing result: not cached
    const bool forced16 = (h->opt.flags & (PPCG_FLAG_SELL_COL16 | PPCG_FLAG_SELL_COL32)) != 0;
    const bool shared = PPCG_SELL_SHARED && !(h->opt.flags & PPCG_FLAG_SELL_NO_SHARED_OFFSETS);
    // Row-length statistics.
    double sum = 0, sum2 = 0;
    int mx = 0;
    for (int v : rowlen_h) {
        sum += v;
        sum2 += (double)v * v;
        mx = std::max(mx, v);
    }
    const double mean = sum / h->n;
    const double var = std::max(0.0, sum2 / h->n - mean * mean);
    const double cv = mean > 0 ? std::sqrt(var) / mean : 0.0;
    auto pow2_near = [](double v) {
        int l = 2;
        while (l < 64 && l < v)
            l <<= 1;
        return l;
    };
    if (want == PPCG_SPMV_SELL) {
        int64_t st1 = 0;
        PPCG_TRY(sell_size(h->stream, h->n, 1, rowlen, &st1));
        const int sigma = (double)st1 > 1.05 * (double)h->nnz ? kSortWindow : 1;
        SellBuild sb;
        PPCG_TRY(build_sell(h->stream, h->n, sigma, rp, ci, val, rowlen, &sb, shared));
        PPCG_TRY(adopt_sell(h, sb));
        PPCG_TRY(bind_f64(h, dinv_orig));
        int c16 = 0;
        return tune_col16(h, -1, &c16);
    }
    if (want == PPCG_SPMV_CSR_VECTOR) {
        PPCG_TRY(adopt_csrv(h, csrv_default_lanes(mean), rp, ci, val));
        return bind_f64(h, dinv_orig);
    }
    TuneKey key{(int)std::log2((double)h->n), (int)std::lround(mean), (int)std::lround(10 * cv),
                (int)std::log2((double)std::max(mx, 1))};
    TuneVal tv{};
    bool hit = false;
    {
        std::unique_lock<std::mutex> lk(g_tune_mu);
        g_tune_cv.wait(lk, [&] { return !g_tuning.count(key); });
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            tv = it->second;
            hit = true;
        } else {
            g_tuning.insert(key);  // this thread tunes the signature
        }
    }
    if (hit) {
        if (tv.fmt == FMT_SELL) {
            SellBuild sb;
            PPCG_TRY(build_sell(h->stream, h->n, tv.sigma, rp, ci, val, rowlen, &sb, shared));
            PPCG_TRY(adopt_sell(h, sb));
        } else {
            PPCG_TRY(adopt_csrv(h, tv.lanes, rp, ci, val));
        }
        PPCG_TRY(bind_f64(h, dinv_orig));
        int c16 = 0;
        PPCG_TRY(tune_col16(h, tv.col16, &c16));
        if (tv.col16 < 0 && !forced16) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key].col16 = c16;  // timed now (the entry came from a forced choice)
        }
        return PPCG_OK;
    }
    // on every return below (the choice stored first on success), the
    // signature is released to the threads waiting for it
    struct Release {
        TuneKey k;
        ~Release()
        {
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tuning.erase(k);
            }
            g_tune_cv.notify_all();
        }
    } release{key};
    struct Cand {
        int fmt, sigma, lanes;
    };
    std::vector<Cand> cands;
    int64_t st1 = 0;
    PPCG_TRY(sell_size(h->stream, h->n, 1, rowlen, &st1));
    cands.push_back({FMT_SELL, 1, 0});
    // rows sorted by length inside windows of sigma rows, when unsorted
    // chunks pad by more than 1 %: every window size is timed
    if ((double)st1 > 1.01 * (double)h->nnz)
        for (int w : kSortWindows)
            if (w < h->n)
                cands.push_back({FMT_SELL, w, 0});
    // CSR-vector with groups of 2 .. 64 lanes around a quarter of the mean
    // row length
    if (mean >= 8.0) {
        const int l = pow2_near(mean / 4);
        for (int lanes : {l / 4, l / 2, l, l * 2, l * 4})
            if (lanes >= 2 && lanes <= 64)
                cands.push_back({FMT_CSRV, 1, lanes});
    }
    double best = 1e300;
    Cand bestc = cands[0];
    for (const Cand &c : cands) {
        if (c.fmt == FMT_SELL) {
            SellBuild sb;
            PPCG_TRY(build_sell(h->stream, h->n, c.sigma, rp, ci, val, rowlen, &sb, shared));
            PPCG_TRY(adopt_sell(h, sb));
        } else {
            PPCG_TRY(adopt_csrv(h, c.lanes, rp, ci, val));
        }
        PPCG_TRY(bind_f64(h, dinv_orig));
        double ms = 0;
        PPCG_TRY(time_spmv(h, 5, &ms));
        if (ms < best) {
            best = ms;
            bestc = c;
        }
    }
    const Cand &last = cands.back();
    if (!(last.fmt == bestc.fmt && last.sigma == bestc.sigma && last.lanes == bestc.lanes)) {
        if (bestc.fmt == FMT_SELL) {
            SellBuild sb;
            PPCG_TRY(build_sell(h->stream, h->n, bestc.sigma, rp, ci, val, rowlen, &sb, shared));
            PPCG_TRY(adopt_sell(h, sb));
        } else {
            PPCG_TRY(adopt_csrv(h, bestc.lanes, rp, ci, val));
        }
    }
    PPCG_TRY(bind_f64(h, dinv_orig));
    int c16 = 0;
    PPCG_TRY(tune_col16(h, -1, &c16));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {bestc.fmt, bestc.sigma, bestc.lanes, forced16 ? -1 : c16};
    }
    return PPCG_OK;
}

// Allocate the FP64 solver vectors and partial sums.
static ppcg_status alloc_f64_vectors(ppcg_handle *h)
{
    const size_t n = (size_t)h->n;
    const size_t vb = aligned(n * sizeof(double));
    const size_t pb = aligned((size_t)2 * h->ntiles * kPartStride * sizeof(double));
    PPCG_TRY(h->f64.arena.alloc(11 * vb + pb + 2 * 256));
    for (int k = 0; k < 11; ++k)
        h->f64.vec[k] = h->f64.arena.take(n * sizeof(double));
    h->part = (double *)h->f64.arena.take((size_t)2 * h->ntiles * kPartStride * sizeof(double));
    return PPCG_OK;
}

// FP32 copy of the stored matrix values (both mixed modes).
ppcg_status ensure_val32(ppcg_handle *h)
{
    if (h->val32)
        return PPCG_OK;
    const size_t m = (size_t)std::max<int64_t>(h->nnz_stored, 1);
    PPCG_HIP(hipMalloc(&h->val32, m * sizeof(float)));
    k_convert<float, double><<<blocks_for((size_t)h->nnz_stored, 256), 256, 0, h->stream>>>(
        (size_t)h->nnz_stored, h->val64, h->val32);
    PPCG_HIP(hipGetLastError());
    PPCG_HIP(hipStreamSynchronize(h->stream));
    return PPCG_OK;
}

// FP32 vectors and values for the FP32 mixed-precision sequence.
ppcg_status ensure_f32(ppcg_handle *h)
{
    if (h->f32.ready)
        return PPCG_OK;
    PPCG_TRY(ensure_val32(h));
    const size_t n = (size_t)h->n;
    const size_t vb = aligned(n * sizeof(float));
    const size_t pb = aligned((size_t)2 * h->ntiles * kPartStride * sizeof(double));
    PrecData &pd = h->f32;
    PPCG_TRY(pd.arena.alloc(12 * vb + pb + 4 * 256));
    pd.prec = PREC_F32;
    pd.val = h->val32;
    pd.dinv = pd.arena.take(n * sizeof(float));
    for (int k = 0; k < 11; ++k)
        pd.vec[k] = pd.arena.take(n * sizeof(float));
    h->part32 = (double *)pd.arena.take((size_t)2 * h->ntiles * kPartStride * sizeof(double));
    k_convert<float, double><<<blocks_for(n, 256), 256, 0, h->stream>>>(n, h->dinv64, (float *)pd.dinv);
    PPCG_HIP(hipGetLastError());
    PPCG_HIP(hipStreamSynchronize(h->stream));
    pd.ready = true;
    return PPCG_OK;
}

// ---------------------------------------------------------------- engine
Engine::~Engine()
{
    for (int k = 0; k < kGroups; ++k) {
        if (gstream_[k]) {
            (void)hipStreamSynchronize(gstream_[k]);
            (void)hipStreamDestroy(gstream_[k]);
        }
        if (ev_join_[k]) (void)hipEventDestroy(ev_join_[k]);
    }
    if (ev_fork_) (void)hipEventDestroy(ev_fork_);
    for (Group *g : {&g64_, &gv_, &gs_, &gp_, &gpv_, &gp32_, &gf_}) {
        drop_graphs(*g);
        if (g->desc_d) (void)dev_free(g->desc_d);
        if (g->st_d) (void)dev_free(g->st_d);
        if (g->st_h) (void)host_free(g->st_h);
        if (g->table_d) (void)dev_free(g->table_d);
        if (g->count_d) (void)dev_free(g->count_d);
        if (g->aux_d) (void)dev_free(g->aux_d);
        if (g->aux_count_d) (void)dev_free(g->aux_count_d);
        if (g->sys_d) (void)dev_free(g->sys_d);
        if (g->sys_count_d) (void)dev_free(g->sys_count_d);
        if (g->stage_h) (void)host_free(g->stage_h);
        if (g->stage_cnt_h) (void)host_free(g->stage_cnt_h);
        if (g->desc_stage_h) (void)host_free(g->desc_stage_h);
    }
    if (ev_desc_) (void)hipEventDestroy(ev_desc_);
}

BatchCtx::~BatchCtx()
{
    delete E;
    if (items_d) (void)dev_free(items_d);
    if (items_h) (void)host_free(items_h);
}

ppcg_status Engine::ensure_group(Group &g, int prec, int cap_sys)
{
    g.prec = prec;
    if (g.cap_sys >= cap_sys)
        return PPCG_OK;
    if (g.cap_sys > 0) {
        set_error("engine capacity is fixed once initialised");
        return PPCG_ERR_INVALID_ARG;
    }
    g.cap_sys = cap_sys;
    PPCG_HIP(hipMalloc(&g.desc_d, sizeof(SysDesc) * cap_sys));
    PPCG_HIP(hipMalloc(&g.st_d, sizeof(SysState) * cap_sys));
    PPCG_HIP(hipHostMalloc((void **)&g.st_h, sizeof(SysState) * cap_sys, hipHostMallocDefault));
    PPCG_HIP(hipMalloc(&g.count_d, sizeof(int)));
    PPCG_HIP(hipMalloc(&g.aux_count_d, sizeof(int)));
    PPCG_HIP(hipMalloc(&g.sys_count_d, sizeof(int)));
    PPCG_HIP(hipHostMalloc((void **)&g.stage_cnt_h, sizeof(int) * 3, hipHostMallocDefault));
    PPCG_HIP(hipHostMalloc((void **)&g.desc_stage_h, sizeof(SysDesc) * cap_sys, hipHostMallocDefault));
    g.desc_h.assign(cap_sys, SysDesc{});
    g.slot_used.assign(cap_sys, 0);
    g.desc_pending.assign(cap_sys, 0);
    g.st_pending.assign(cap_sys, 0);
    // never equal to a filled descriptor (n >= 1), so the first upload happens
    SysDesc none;
    memset(&none, 0, sizeof none);
    g.desc_up.assign(cap_sys, none);
    return PPCG_OK;
}

ppcg_status Engine::init(int cap_sys)
{
    if (!ev_fork_) {
        PPCG_HIP(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
        PPCG_HIP(hipEventCreateWithFlags(&ev_desc_, hipEventDisableTiming));
        for (int k = 0; k < kGroups; ++k) {
            PPCG_HIP(hipStreamCreateWithFlags(&gstream_[k], hipStreamNonBlocking));
            PPCG_HIP(hipEventCreateWithFlags(&ev_join_[k], hipEventDisableTiming));
        }
    }
    PPCG_TRY(ensure_group(g64_, PREC_F64, cap_sys));
    PPCG_TRY(ensure_group(gv_, PREC_V32, cap_sys));
    PPCG_TRY(ensure_group(gs_, PREC_F64, cap_sys));
    PPCG_TRY(ensure_group(gp_, PREC_F64, cap_sys));
    PPCG_TRY(ensure_group(gpv_, PREC_V32, cap_sys));
    PPCG_TRY(ensure_group(gp32_, PREC_F32, cap_sys));
    PPCG_TRY(ensure_group(gf_, PREC_F64, cap_sys));
    gp_.pcg = gpv_.pcg = gp32_.pcg = true;
    gf_.fused = true;
    return PPCG_OK;
}

int Engine::alloc_slot(Group &g)
{
    for (int i = 0; i < g.cap_sys; ++i)
        if (!g.slot_used[i]) {
            g.slot_used[i] = 1;
            return i;
        }
    return -1;
}

ppcg_status Engine::upload_desc(Group &g, int slot)
{
    // descriptors are built from a zeroed record (padding included), so an
    // unchanged one compares equal byte for byte and is not sent again
    if (memcmp(&g.desc_up[slot], &g.desc_h[slot], sizeof(SysDesc)) == 0)
        return PPCG_OK;
    g.desc_pending[slot] = 1;
    g.desc_up[slot] = g.desc_h[slot];
    return PPCG_OK;
}

// Send the queued descriptor uploads (through the group's pinned staging,
// one copy per run of consecutive slots) and state clears.  Adding a batch
// of systems thus costs a few transfers instead of two per system.
ppcg_status Engine::flush_uploads()
{
    Group *const groups[] = {&g64_, &gv_, &gs_, &gp_, &gpv_, &gp32_, &gf_};
    bool copies = false;
    for (Group *g : groups) {
        for (int a = 0; a < g->cap_sys;) {
            if (!g->desc_pending[a]) {
                ++a;
                continue;
            }
            int b = a;
            while (b < g->cap_sys && g->desc_pending[b])
                g->desc_pending[b++] = 0;
            if (!copies && desc_copy_queued_) {
                // the staging may still feed the previous flush's copies
                PPCG_HIP(hipEventSynchronize(ev_desc_));
                desc_copy_queued_ = false;
            }
            copies = true;
            memcpy(g->desc_stage_h + a, &g->desc_h[a], sizeof(SysDesc) * (b - a));
            PPCG_HIP(hipMemcpyAsync(g->desc_d + a, g->desc_stage_h + a, sizeof(SysDesc) * (b - a),
                                    hipMemcpyHostToDevice, stream_));
            a = b;
        }
        for (int a = 0; a < g->cap_sys;) {
            if (!g->st_pending[a]) {
                ++a;
                continue;
            }
            int b = a;
            while (b < g->cap_sys && g->st_pending[b])
                g->st_pending[b++] = 0;
            PPCG_HIP(hipMemsetAsync(g->st_d + a, 0, sizeof(SysState) * (b - a), stream_));
            a = b;
        }
    }
    if (copies) {
        PPCG_HIP(hipEventRecord(ev_desc_, stream_));
        desc_copy_queued_ = true;
    }
    return PPCG_OK;
}

static ppcg_status grow_table(WorkItem **d, int *cap, int need)
{
    if (*cap >= need)
        return PPCG_OK;
    int nc = std::max(need, *cap * 2);
    nc = std::max(nc, 64);
    if (*d)
        (void)dev_free(*d);
    *d = nullptr;
    PPCG_HIP(hipMalloc(d, sizeof(WorkItem) * nc));
    *cap = nc;
    return PPCG_OK;
}

// Upload a work table through the pinned staging buffer.  The caller has
// synchronised the stream since the staging buffer was last used.
static ppcg_status upload_table(hipStream_t s, Group &g, const std::vector<WorkItem> &items, WorkItem *dst,
                                int *cnt_d, int which)
{
    const int n = (int)items.size();
    if (g.stage_cap < n + 1) {
        if (g.stage_h)
            (void)host_free(g.stage_h);
        g.stage_h = nullptr;
        g.stage_cap = std::max(2 * n + 1, 256);
        // three regions: iteration table, aux table, system table
        PPCG_HIP(hipHostMalloc((void **)&g.stage_h, sizeof(WorkItem) * g.stage_cap * 3, hipHostMallocDefault));
    }
    WorkItem *st = g.stage_h + (size_t)which * g.stage_cap;
    if (n)
        memcpy(st, items.data(), sizeof(WorkItem) * n);
    g.stage_cnt_h[which] = n;
    if (n)
        PPCG_HIP(hipMemcpyAsync(dst, st, sizeof(WorkItem) * n, hipMemcpyHostToDevice, s));
    PPCG_HIP(hipMemcpyAsync(cnt_d, &g.stage_cnt_h[which], sizeof(int), hipMemcpyHostToDevice, s));
    return PPCG_OK;
}

// Launch sequences of FP64 Algorithm 2 over a work table, shared by the
// engine and ppcg_solve_noalloc.
void launch_x_complete(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid)
{
    k_x_fixup<double><<<grid, 256, 0, s>>>(tab, cnt, dd);
    k_x_settle<<<grid, 64, 0, s>>>(tab, cnt, dd);
}

void launch_pipecg_init(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid, bool x_zero)
{
    const int rs = PPCG_XCD_REMAP_SPMV;
    if (x_zero)
        k_spmv<double, MODE_INIT0><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
    else
        k_spmv<double, MODE_INIT1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
    k_spmv<double, MODE_INIT2><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
    k_spmv<double, MODE_ITER><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
}

void launch_pipecg_iter(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid, int remap)
{
    k_vma<double><<<grid, kVmaThreads, 0, s>>>(tab, cnt, dd, remap);
    k_spmv<double, MODE_ITER><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, PPCG_XCD_REMAP_SPMV);
}

void launch_pipecg_init_fused(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid,
                              bool x_zero)
{
    const int rs = PPCG_XCD_REMAP_SPMV;
    if (x_zero)
        k_spmv<double, MODE_INIT0><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
    else
        k_spmv<double, MODE_INIT1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
    k_spmv<double, MODE_INIT2><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
}

void launch_fused_chunk(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid, int iters)
{
    k_fused_begin<<<grid, 64, 0, s>>>(tab, cnt, dd);
    for (int i = 0; i < iters; ++i)
        k_fused<<<grid, kFusedThreads, 0, s>>>(tab, cnt, dd, PPCG_FUSED_REMAP, i & 1);
}

void launch_true_resid(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid)
{
    k_spmv<double, MODE_RESID><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, PPCG_XCD_REMAP_SPMV);
    k_reduce_resid<<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd);
}

void launch_validate(hipStream_t s, int n, int64_t nnz, const int *rp, const int *ci, const double *val,
                     double *dinv, int *rowlen, unsigned *err)
{
    k_validate<<<blocks_for(n, 256), 256, 0, s>>>(n, nnz, rp, ci, val, dinv, rowlen, err);
}

void set_csr_error(const unsigned (&err)[2])
{
    std::string what;
    const char *names[] = {"row_ptr[0] != 0", "row_ptr[n] != nnz", "row_ptr not monotone / out of range",
                           "column index out of range", "columns not strictly ascending",
                           "missing diagonal", "diagonal not positive", "non-finite value"};
    for (int b = 0; b < 8; ++b)
        if (err[0] & (1u << b)) {
            if (!what.empty())
                what += ", ";
            what += names[b];
        }
    set_error("bad CSR: %s (first row %u)", what.c_str(), err[1]);
}

// One iteration of a group: the fused update, then the SpMV with the
// in-launch reduction.  The FP32-values group uses the fused-update variant
// that also emits the direct-denominator partials.
static void launch_iter_pair(hipStream_t s, const Group &g, int grid, int remap)
{
    if (g.pcg) {
        // Algorithm 1: SpMV, alpha, vector updates, stopping test and beta.
        const int sg = std::max(g.g_sys_grid, 1);
        if (g.prec == PREC_F32)
            k_pcg_spmv<float><<<grid, kSpmvThreads, 0, s>>>(g.table_d, g.count_d, g.desc_d, PPCG_XCD_REMAP_SPMV);
        else
            k_pcg_spmv<double><<<grid, kSpmvThreads, 0, s>>>(g.table_d, g.count_d, g.desc_d, PPCG_XCD_REMAP_SPMV);
        k_pcg_alpha<<<sg, kPcgRedThreads, 0, s>>>(g.sys_d, g.sys_count_d, g.desc_d);
        if (g.prec == PREC_F32)
            k_pcg_vma<float><<<grid, kVmaThreads, 0, s>>>(g.table_d, g.count_d, g.desc_d, remap);
        else
            k_pcg_vma<double><<<grid, kVmaThreads, 0, s>>>(g.table_d, g.count_d, g.desc_d, remap);
        k_pcg_update<PCG_ITER><<<sg, kPcgRedThreads, 0, s>>>(g.sys_d, g.sys_count_d, g.desc_d);
    } else if (g.prec == PREC_V32) {
        k_vma<double, true><<<grid, kVmaThreads, 0, s>>>(g.table_d, g.count_d, g.desc_d, remap);
        k_spmv<double, MODE_ITER><<<grid, kSpmvThreads, 0, s>>>(g.table_d, g.count_d, g.desc_d, PPCG_XCD_REMAP_SPMV);
    } else {
        launch_pipecg_iter(s, g.table_d, g.count_d, g.desc_d, grid, remap);
    }
}

ppcg_status Engine::ensure_table(Group &g)
{
    if (!g.table_dirty)
        return PPCG_OK;
    // the table on the device is already this one (e.g. the same system
    // solved again after its table emptied on the host): nothing to send,
    // and no wait for the staging buffer
    if (g.table_h.size() == g.table_up.size() &&
        std::equal(g.table_h.begin(), g.table_h.end(), g.table_up.begin(),
                   [](const WorkItem &a, const WorkItem &b) { return a.slot == b.slot && a.tile == b.tile; })) {
        g.table_dirty = false;
        return PPCG_OK;
    }
    PPCG_HIP(hipStreamSynchronize(stream_));  // table_d / staging may still be in use
    WorkItem *old = g.table_d;
    PPCG_TRY(grow_table(&g.table_d, &g.table_cap, (int)g.table_h.size()));
    if (old != g.table_d)  // graphs baked the old pointer
        drop_graphs(g);
    PPCG_TRY(upload_table(stream_, g, g.table_h, g.table_d, g.count_d, 0));
    if (g.pcg) {
        std::vector<WorkItem> sys;
        for (const WorkItem &w : g.table_h)
            if (w.tile == 0)
                sys.push_back(w);
        WorkItem *olds = g.sys_d;
        PPCG_TRY(grow_table(&g.sys_d, &g.sys_cap, (int)sys.size()));
        if (olds != g.sys_d)
            drop_graphs(g);
        PPCG_TRY(upload_table(stream_, g, sys, g.sys_d, g.sys_count_d, 2));
        g.nsys = (int)sys.size();
    }
    g.table_up = g.table_h;
    g.table_dirty = false;
    return PPCG_OK;
}

void Engine::drop_graphs(Group &g)
{
    for (auto &kv : g.graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    g.graphs.clear();
    g.g_grid = 0;
    g.g_sys_grid = 0;
}

// Graph of `iters` iterations over the group's table.  The grid is baked
// into the graph; workgroups past the live table size exit at once, so a
// graph stays valid while the table shrinks, and graphs are recaptured when
// the table outgrows the grid or shrinks below a quarter of it.
ppcg_status Engine::ensure_graph(Group &g, int iters, hipGraphExec_t *exec)
{
    const int need = std::max((int)g.table_h.size(), 1);
    const int need_sys = std::max(g.nsys, 1);
    if (g.g_grid < need || g.g_grid > std::max(need * 4, 64) ||
        (g.pcg && (g.g_sys_grid < need_sys || g.g_sys_grid > std::max(need_sys * 4, 16))))
        drop_graphs(g);
    auto it = g.graphs.find(iters);
    if (it != g.graphs.end()) {
        *exec = it->second.exec;
        return PPCG_OK;
    }
    const int grid = g.g_grid ? g.g_grid : need;
    if (g.pcg && !g.g_sys_grid)
        g.g_sys_grid = need_sys;
    std::unique_lock<std::shared_mutex> no_release(release_mu());
    Group::CapturedGraph cg;
    PPCG_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    if (g.fused)
        launch_fused_chunk(stream_, g.table_d, g.count_d, g.desc_d, grid, iters);
    else
        for (int i = 0; i < iters; ++i)
            launch_iter_pair(stream_, g, grid, remap);
    hipError_t e = hipStreamEndCapture(stream_, &cg.graph);
    if (e != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return PPCG_ERR_DEVICE;
    }
    e = hipGraphInstantiate(&cg.exec, cg.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(cg.graph);
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return PPCG_ERR_DEVICE;
    }
    g.g_grid = grid;
    g.graphs[iters] = cg;
    *exec = cg.exec;
    return PPCG_OK;
}

// Iterations for the next chunk of a group: the most any of its iterating
// jobs still needs (exact in fixed-iteration mode, predicted from the
// observed convergence rate otherwise), capped at max_iters and rounded down
// to a power of two so that few graphs are ever captured.
int iters_needed(const SysDesc &d, const SysState &st, double rate, bool polled, int max_iters, bool pcg)
{
    int rem = max_iters;
    if (d.fixed > 0) {
        rem = d.fixed - (polled ? st.iter : 0);
    } else if (polled && rate > 0.0 && rate < 0.9999) {
        const double cur = d.stop == STOP_ABS ? std::sqrt(st.uu) : std::sqrt(st.rr);
        double target = d.stop == STOP_ABS ? d.tol : d.tol * std::sqrt(st.bnorm2);
        // a classic-PCG sequence that pauses for reliable updates stops at
        // the pause if that comes first
        if (pcg && d.repl_factor > 0.0 && d.stop == STOP_REL)
            target = std::max(target, d.repl_factor * st.repl_ref);
        if (cur > target && target > 0.0)
            rem = (int)std::ceil(1.1 * std::log(target / cur) / std::log(rate)) + 1;
    }
    return std::max(1, std::min(rem, max_iters));
}

void note_progress(const SysDesc &d, const SysState &st, double *last_norm, int *last_iter, double *rate)
{
    const double cur = d.stop == STOP_ABS ? std::sqrt(st.uu) : std::sqrt(st.rr);
    if (*last_norm > 0 && st.iter > *last_iter)
        *rate = std::pow(cur / *last_norm, 1.0 / (st.iter - *last_iter));
    *last_norm = cur;
    *last_iter = st.iter;
}

int Engine::chunk_iters(const Group &g, int max_iters)
{
    int want = 1;
    for (const Job &j : jobs_) {
        if (j.finished || j.stage != JS_ITER || &pgroup(j) != &g)
            continue;
        want = std::max(want, iters_needed(g.desc_h[pslot(j)], g.st_h[pslot(j)], j.rate, j.last_norm >= 0,
                                           max_iters, g.pcg));
    }
    // The single-launch form: its first launch after an initialisation does
    // no update, so k updates take k + 1 launches, and chunks hold an even
    // number of launches (the parity of m, partials and state returns to 0).
    if (g.fused)
        want = std::max(2, std::min(want + 1, std::max(max_iters, 2)));
    int k = 1;
    while (k * 2 <= want)
        k *= 2;
    return k;
}

std::vector<int> Engine::chunk_plan(const Group &g, int max_iters, bool *covers)
{
    *covers = false;
    bool all_fixed = true;
    int want = 1;
    for (const Job &j : jobs_) {
        if (j.finished || j.stage != JS_ITER || &pgroup(j) != &g)
            continue;
        const SysDesc &d = g.desc_h[pslot(j)];
        if (d.fixed <= 0 || d.repl_factor > 0.0)
            all_fixed = false;
        want = std::max(want, iters_needed(d, g.st_h[pslot(j)], j.rate, j.last_norm >= 0, INT_MAX / 4, g.pcg));
    }
    if (!all_fixed || g.pcg)
        return {chunk_iters(g, max_iters)};
    int cap = 1;
    while (cap * 2 <= max_iters)
        cap *= 2;
    if (g.fused) {
        // k updates take k + 1 launches, an even number per chunk
        want += 1;
        want += want & 1;
        cap = std::max(cap, 2);
    }
    int left = std::min(want, kFixedChunksPerPoll * cap);
    *covers = left == want;
    // a run that fits one chunk gets a graph of its exact length (one graph
    // per fixed-iteration count): no launch gap and chunk-start node between
    // chunks of powers of two
    if (left <= cap)
        return {left};
    std::vector<int> plan;
    while (left > 0) {
        int c = 1;
        while (c * 2 <= left && c * 2 <= cap)
            c *= 2;
        if (g.fused && c < 2)
            c = 2;
        plan.push_back(c);
        left -= c;
    }
    return plan;
}

ppcg_status Engine::sync_states(Group &g)
{
    PPCG_HIP(hipMemcpyAsync(g.st_h, g.st_d, sizeof(SysState) * g.cap_sys, hipMemcpyDeviceToHost, stream_));
    return PPCG_OK;
}

// Run an auxiliary operation over all tiles of the given slots of group g.
ppcg_status Engine::aux_launch(Group &g, const std::vector<int> &slots, int what, const Group *inner)
{
    if (slots.empty())
        return PPCG_OK;
    PPCG_TRY(flush_uploads());
    std::vector<WorkItem> items;
    for (int sl : slots)
        for (int t = 0; t < g.desc_h[sl].ntiles; ++t)
            items.push_back({sl, t});
    const bool same = items.size() == g.aux_h.size() &&
                      std::equal(items.begin(), items.end(), g.aux_h.begin(),
                                 [](const WorkItem &a, const WorkItem &b) { return a.slot == b.slot && a.tile == b.tile; });
    if (!same) {
        // The staging buffer and aux_d may still be read by earlier enqueued
        // copies and kernels: drain the stream before reusing them.
        PPCG_HIP(hipStreamSynchronize(stream_));
        WorkItem *old = g.aux_d;
        PPCG_TRY(grow_table(&g.aux_d, &g.aux_cap, (int)items.size()));
        (void)old;
        PPCG_TRY(upload_table(stream_, g, items, g.aux_d, g.aux_count_d, 1));
        g.aux_h = items;
    }
    const int grid = (int)items.size();
    hipStream_t s = stream_;
    const WorkItem *tab = g.aux_d;
    const int *cnt = g.aux_count_d;
    const SysDesc *dd = g.desc_d;
    const int rs = PPCG_XCD_REMAP_SPMV;
    const bool f32 = g.prec == PREC_F32;
    // the fused update of Algorithm 2 defers every other x-update: complete
    // x before anything reads it (a no-op for systems with nothing pending)
    // (the single-launch form applies a deferred x-update in the launch that
    // stops the system, so its x is always complete here)
    if (!g.pcg && !g.fused && &g != &gs_ && (what == AUX_RESID || what == AUX_REPL || what == AUX_INIT))
        launch_x_complete(s, tab, cnt, dd, grid);
    const bool x_zero = what == AUX_START0;
    if (what == AUX_START || what == AUX_START0)  // a first start: nothing deferred, x complete
        what = AUX_INIT;
    if (what == AUX_INIT && g.pcg) {
        if (f32) {
            k_spmv<float, MODE_INIT1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
            k_pcg_dots<float><<<grid, kVmaThreads, 0, s>>>(tab, cnt, dd);
        } else {
            if (x_zero)
                k_spmv<double, MODE_INIT0><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
            else
                k_spmv<double, MODE_INIT1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
            k_pcg_dots<double><<<grid, kVmaThreads, 0, s>>>(tab, cnt, dd);
        }
        k_pcg_update<PCG_START><<<grid, kPcgRedThreads, 0, s>>>(tab, cnt, dd);
    } else if (what == AUX_REPL && g.pcg) {
        // Reliable update of classic PCG: r = b - A x, u = M^-1 r; p is kept.
        // FP64 vectors use the FP64 values; the FP32 mixed-precision slots
        // recompute their FP32 residual of the rescaled system (x32 = 0).
        if (f32) {
            k_spmv<float, MODE_REPL1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
            k_pcg_dots<float><<<grid, kVmaThreads, 0, s>>>(tab, cnt, dd);
        } else {
            k_spmv<double, MODE_REPL1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
            k_pcg_dots<double><<<grid, kVmaThreads, 0, s>>>(tab, cnt, dd);
        }
        k_pcg_update<PCG_REPL><<<grid, kPcgRedThreads, 0, s>>>(tab, cnt, dd);
    } else if (what == AUX_INIT && g.fused) {
        launch_pipecg_init_fused(s, tab, cnt, dd, grid, x_zero);
    } else if (what == AUX_INIT) {
        launch_pipecg_init(s, tab, cnt, dd, grid, x_zero);
    } else if (what == AUX_RESID) {
        launch_true_resid(s, tab, cnt, dd, grid);
    } else if (what == AUX_REPL) {
        // Reliable update: FP64 residual, then the rebuilt auxiliaries (two
        // dual-product passes with the iteration's values).
        k_spmv<double, MODE_REPL1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
        k_spmv<double, MODE_DUAL1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
        k_spmv<double, MODE_DUAL2><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, rs);
    } else if (what == AUX_MIX_START) {
        k_pcg_mix_start<<<grid, 256, 0, s>>>(tab, cnt, g64_.desc_d, inner->desc_d);
    } else if (what == AUX_MIX_CORRECT) {
        k_pcg_mix_correct<<<grid, 256, 0, s>>>(tab, cnt, g64_.desc_d, inner->desc_d);
    }
    PPCG_HIP(hipGetLastError());
    return PPCG_OK;
}

ppcg_status Engine::add(ppcg_handle *h, int mixed, double tol, const double *, int *job_id)
{
    Job j;
    j.h = h;
    j.mixed = mixed;
    j.tol = tol;
    j.x0_zero = h->x0_zero;
    j.t_start = now_ms();
    const ppcg_options &o = h->opt;
    const int stop = o.stop == PPCG_STOP_PRECOND_ABS ? STOP_ABS : STOP_REL;
    auto release = [&]() {
        if (j.slot64 >= 0) g64_.slot_used[j.slot64] = 0;
        if (j.slot32 >= 0) gp32_.slot_used[j.slot32] = 0;
        if (j.slotv >= 0) gv_.slot_used[j.slotv] = 0;
    };
    auto fail = [&](ppcg_status s) {
        release();
        return s;
    };
    // FP32 vectors always iterate with Algorithm 1: the pipelined method's
    // auxiliary recurrences (w, z, s) drift away from A u, A q, A p within a
    // few dozen FP32 iterations, even with the other vectors recomputed
    if (o.method == PPCG_METHOD_PCG || mixed == MIX_INNER32)
        j.pcg = true;
    if (j.pcg && mixed != MIX_INNER32) {
        const bool v32 = mixed == MIX_VALUES32;
        Group &g = v32 ? gpv_ : gp_;
        int &slot = v32 ? j.slotv : j.slot64;
        slot = alloc_slot(g);
        if (slot < 0) {
            set_error("engine has no free slot");
            return PPCG_ERR_INVALID_ARG;
        }
        ppcg_status rc = v32 ? ensure_val32(h) : PPCG_OK;
        if (rc == PPCG_OK)
            rc = fill_desc(h, PREC_F64, g.st_d + slot, &g.desc_h[slot], tol, o.fixed_iters, o.max_iter, stop,
                           v32 ? 1 : 0);
        if (rc != PPCG_OK) {
            g.slot_used[slot] = 0;
            return rc;
        }
        if (v32)
            g.desc_h[slot].repl_factor = o.inner_tol > 0 ? o.inner_tol : 1e-3;
        PPCG_TRY(upload_desc(g, slot));
        clear_state(g, slot);
        j.stage = JS_NEED_INIT;
    } else if (mixed == MIX_VALUES32) {
        j.slotv = alloc_slot(gv_);
        if (j.slotv < 0) {
            set_error("engine has no free slot");
            return PPCG_ERR_INVALID_ARG;
        }
        ppcg_status rc = ensure_val32(h);
        if (rc == PPCG_OK)
            rc = fill_desc(h, PREC_F64, gv_.st_d + j.slotv, &gv_.desc_h[j.slotv], tol, o.fixed_iters, o.max_iter,
                           stop, 1);
        if (rc != PPCG_OK)
            return fail(rc);
        gv_.desc_h[j.slotv].repl_factor = o.inner_tol > 0 ? o.inner_tol : 1e-3;
        PPCG_TRY(upload_desc(gv_, j.slotv));
        clear_state(gv_, j.slotv);
        j.stage = JS_NEED_INIT;
    } else if (mixed == MIX_NONE && h->form == FORM_FUSED && h->frec && h->fmt == FMT_SELL) {
        j.fused = true;
        j.slot64 = alloc_slot(gf_);
        if (j.slot64 < 0) {
            set_error("engine has no free slot");
            return PPCG_ERR_INVALID_ARG;
        }
        ppcg_status rc = fill_desc(h, PREC_F64, gf_.st_d + j.slot64, &gf_.desc_h[j.slot64], tol, o.fixed_iters,
                                   o.max_iter, stop);
        if (rc != PPCG_OK) {
            gf_.slot_used[j.slot64] = 0;
            return rc;
        }
        PPCG_TRY(upload_desc(gf_, j.slot64));
        clear_state(gf_, j.slot64);
        j.stage = JS_NEED_INIT;
    } else if (mixed == MIX_NONE && h->fmt == FMT_SELL && h->n <= PPCG_SMALL_MAX_ROWS) {
        j.small = true;
        j.slot64 = alloc_slot(gs_);
        if (j.slot64 < 0) {
            set_error("engine has no free slot");
            return PPCG_ERR_INVALID_ARG;
        }
        ppcg_status rc = fill_desc(h, PREC_F64, gs_.st_d + j.slot64, &gs_.desc_h[j.slot64], tol, o.fixed_iters,
                                   o.max_iter, stop);
        if (rc != PPCG_OK) {
            gs_.slot_used[j.slot64] = 0;
            return rc;
        }
        PPCG_TRY(upload_desc(gs_, j.slot64));
        clear_state(gs_, j.slot64);
        j.stage = JS_NEED_INIT;
    } else {
        j.slot64 = alloc_slot(g64_);
        if (j.slot64 < 0) {
            set_error("engine has no free slot");
            return PPCG_ERR_INVALID_ARG;
        }
        ppcg_status rc = fill_desc(h, PREC_F64, g64_.st_d + j.slot64, &g64_.desc_h[j.slot64], tol,
                                   mixed == MIX_INNER32 ? 0 : o.fixed_iters, o.max_iter, stop);
        if (rc != PPCG_OK)
            return fail(rc);
        if (mixed == MIX_INNER32) {
            rc = ensure_f32(h);
            if (rc != PPCG_OK)
                return fail(rc);
            // the FP32 sequence (Algorithm 1)
            Group &gi = gp32_;
            j.slot32 = alloc_slot(gi);
            if (j.slot32 < 0) {
                set_error("engine has no free slot");
                return fail(PPCG_ERR_INVALID_ARG);
            }
            // its own stop (the FP64 target in the units of the current
            // scaling) is set at every start; it pauses for a reliable update
            // whenever its residual fell by inner_tol
            rc = fill_desc(h, PREC_F32, gi.st_d + j.slot32, &gi.desc_h[j.slot32], tol, 0, o.max_iter, STOP_REL);
            if (rc != PPCG_OK)
                return fail(rc);
            gi.desc_h[j.slot32].repl_factor = o.inner_tol > 0 ? o.inner_tol : kPcgMixReplFactor;
            gi.desc_h[j.slot32].pair = j.slot64;
            g64_.desc_h[j.slot64].pair = j.slot32;
            PPCG_TRY(upload_desc(gi, j.slot32));
            clear_state(gi, j.slot32);
            j.stage = JS_OUTER;
        } else {
            j.stage = JS_NEED_INIT;
        }
        PPCG_TRY(upload_desc(g64_, j.slot64));
        // A new solve starts from a clean state (iteration counters at zero).
        clear_state(g64_, j.slot64);
    }
    jobs_.push_back(j);
    *job_id = (int)jobs_.size() - 1;
    return PPCG_OK;
}

bool Engine::all_done() const
{
    for (const Job &j : jobs_)
        if (!j.finished)
            return false;
    return true;
}

int Engine::active() const
{
    int a = 0;
    for (const Job &j : jobs_)
        a += !j.finished;
    return a;
}

void Engine::reset()
{
    for (int i = 0; i < (int)jobs_.size(); ++i)
        if (jobs_[i].h)
            retire(i);
    jobs_.clear();
}

void Engine::retire(int id)
{
    Job &j = jobs_[id];
    if (j.slot64 >= 0)
        (j.pcg && j.mixed != MIX_INNER32 ? gp_ : j.small ? gs_ : j.fused ? gf_ : g64_).slot_used[j.slot64] = 0;
    if (j.slot32 >= 0)
        gp32_.slot_used[j.slot32] = 0;
    if (j.slotv >= 0)
        (j.pcg ? gpv_ : gv_).slot_used[j.slotv] = 0;
    j.slot64 = j.slot32 = j.slotv = -1;
    j.h = nullptr;
}

static void finish(Job &j, int status, const SysState &st)
{
    j.finished = true;
    j.stage = JS_DONE;
    j.status = status;
    j.t_end = now_ms();
    if (j.mixed != MIX_INNER32) {
        j.iters = st.iter;
        j.bnorm2 = st.bnorm2;
        const double bn = std::sqrt(st.bnorm2);
        j.rel_recur = bn > 0 ? std::sqrt(st.rr) / bn : std::sqrt(st.rr);
        j.precond_norm = std::sqrt(st.uu);
    }
}

// Iterations per launch of the one-workgroup kernel (a few milliseconds).
constexpr int kSmallChunkIters = 512;

ppcg_status Engine::step(int graph_iters)
{
    PPCG_TRY(flush_uploads());
    // 1. Jobs that need a true residual: stopped FP64 / FP32-values jobs, and
    //    FP32-vector jobs at a pause of their sequence (after adding the correction).
    Group *const groups[] = {&g64_, &gv_, &gs_, &gp_, &gpv_, &gp32_, &gf_};
    std::map<Group *, std::vector<int>> resid;  // slots per group
    std::vector<int> correct64;                 // FP64 slots of FP32-vector jobs
    for (Job &j : jobs_) {
        if (j.finished)
            continue;
        if (j.stage == JS_NEED_FINAL)
            resid[&pgroup(j)].push_back(pslot(j));
        else if (j.stage == JS_OUTER) {
            if (j.outer > 0)
                correct64.push_back(j.slot64);
            resid[&g64_].push_back(j.slot64);
        }
    }
    if (!resid.empty()) {
        PPCG_TRY(aux_launch(g64_, correct64, AUX_MIX_CORRECT, &gp32_));
        for (Group *g : groups)
            if (resid.count(g)) {
                PPCG_TRY(aux_launch(*g, resid[g], AUX_RESID));
                PPCG_TRY(sync_states(*g));
            }
        PPCG_HIP(hipStreamSynchronize(stream_));
        // FP64 slots of FP32-vector jobs: sequences to start, and sequences
        // that continue after a reliable update
        std::vector<int> start_mix, repl_mix;
        for (Job &j : jobs_) {
            if (j.finished || (j.stage != JS_NEED_FINAL && j.stage != JS_OUTER))
                continue;
            const SysState &st = j.stage == JS_OUTER ? g64_.st_h[j.slot64] : pgroup(j).st_h[pslot(j)];
            const double bn = std::sqrt(st.bnorm2);
            const double rel = bn > 0 ? std::sqrt(st.tnorm2) / bn : std::sqrt(st.tnorm2);
            j.rel_true = rel;
            const ppcg_options &o = j.h->opt;
            const bool tol_mode = o.fixed_iters <= 0;
            if (j.stage == JS_NEED_FINAL && j.mixed == MIX_VALUES32) {
                // The recurrences follow the FP32-valued operator: a true
                // residual above tol is fixed by a reliable update, not a restart.
                const bool bad = tol_mode && o.stop == PPCG_STOP_REL_RESID && rel > j.tol;
                const bool can_replace = tol_mode && j.outer < o.max_outer && st.iter < o.max_iter;
                if ((st.status == ST_OK && bad) || (st.status == ST_BREAKDOWN && st.i_start > 0)) {
                    if (can_replace) {
                        j.stage = JS_NEED_REPL;
                        continue;
                    }
                    finish(j, st.status == ST_OK ? PPCG_STAGNATED : st.status, st);
                } else {
                    finish(j, st.status, st);
                }
            } else if (j.stage == JS_NEED_FINAL) {
                const FinalAction act = final_action(o, st, j.restarts, rel, j.tol);
                if (act == FINAL_RESTART) {
                    ++j.restarts;
                    j.stage = JS_NEED_INIT;
                    continue;
                }
                finish(j, act == FINAL_STAGNATED ? PPCG_STAGNATED : st.status, st);
            } else {  // FP32-vector mixed precision: outer refinement step
                j.bnorm2 = st.bnorm2;
                if (rel <= j.tol) {
                    finish(j, PPCG_OK, st);
                    j.iters = j.inner_iters;
                    j.rel_recur = rel;
                } else if (j.outer >= o.max_outer || j.inner_iters >= o.max_iter || !(rel == rel)) {
                    finish(j, !(rel == rel) ? PPCG_BREAKDOWN : PPCG_NOT_CONVERGED, st);
                    j.iters = j.inner_iters;
                    j.rel_recur = rel;
                } else {
                    // the sequence continues (its counter runs on); it stops
                    // by itself where the FP64 residual would reach tol:
                    // ||r32|| <= tol ||b|| / ||r64|| on b32 = r64 / ||r64||
                    gp32_.desc_h[j.slot32].tol = j.tol * bn / std::sqrt(st.tnorm2);
                    (j.outer > 0 ? repl_mix : start_mix).push_back(j.slot64);
                    PPCG_TRY(upload_desc(gp32_, j.slot32));
                    j.stage = JS_ITER;
                    ++j.outer;
                }
            }
        }
        // the slot state was cleared when the job was added, so a first
        // start finds no live direction to rescale
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<int> &sl64 = pass == 0 ? start_mix : repl_mix;
            if (sl64.empty())
                continue;
            PPCG_TRY(aux_launch(g64_, sl64, AUX_MIX_START, &gp32_));
            std::vector<int> s32;
            for (int sl : sl64)
                s32.push_back(g64_.desc_h[sl].pair);
            PPCG_TRY(aux_launch(gp32_, s32, pass == 0 ? AUX_INIT : AUX_REPL));
        }
    }
    // 2. Initialisations and reliable updates.
    {
        std::map<Group *, std::vector<int>> init, start, start0, repl;
        for (Job &j : jobs_) {
            if (j.finished)
                continue;
            if (j.stage == JS_NEED_INIT) {
                (j.started ? init : j.x0_zero ? start0 : start)[&pgroup(j)].push_back(pslot(j));
                j.started = true;
                j.stage = JS_ITER;
            } else if (j.stage == JS_NEED_REPL) {
                Group &g = pgroup(j);
                repl[&g].push_back(j.slotv);
                j.stage = JS_ITER;
                ++j.outer;
                if (j.outer >= j.h->opt.max_outer && g.desc_h[j.slotv].repl_factor > 0.0) {
                    // budget spent: no further pauses, iterate to the end
                    g.desc_h[j.slotv].repl_factor = 0.0;
                    PPCG_TRY(upload_desc(g, j.slotv));
                }
            }
        }
        for (Group *g : groups) {
            if (start.count(g))
                PPCG_TRY(aux_launch(*g, start[g], AUX_START));
            if (start0.count(g))
                PPCG_TRY(aux_launch(*g, start0[g], AUX_START0));
            if (init.count(g))
                PPCG_TRY(aux_launch(*g, init[g], AUX_INIT));
            if (repl.count(g))
                PPCG_TRY(aux_launch(*g, repl[g], AUX_REPL));
        }
    }
    // 3. Iteration tables (one work item per system in the small group).
    for (Group *g : groups) {
        std::vector<WorkItem> items;
        for (const Job &j : jobs_) {
            if (j.finished || j.stage != JS_ITER || &pgroup(j) != g)
                continue;
            const int sl = pslot(j);
            const int nt = g == &gs_ ? 1 : g->fused ? g->desc_h[sl].nftiles : g->desc_h[sl].ntiles;
            for (int t = 0; t < nt; ++t)
                items.push_back({sl, t});
        }
        if (items.size() != g->table_h.size() ||
            !std::equal(items.begin(), items.end(), g->table_h.begin(),
                        [](const WorkItem &a, const WorkItem &b) { return a.slot == b.slot && a.tile == b.tile; })) {
            g->table_h = items;
            g->table_dirty = true;
        }
    }
    // 4. One graph chunk per non-empty group, each on its own stream; the
    //    small group runs its chunk as a single launch of the one-workgroup
    //    kernel.  Tables and graphs are prepared on stream_ first.
    std::vector<hipGraphExec_t> execs[kGroups];
    int small_iters = 0;
    std::vector<Group *> finals;  // groups whose fixed-iteration jobs all end in this step
    for (int k = 0; k < kGroups; ++k) {
        Group *g = groups[k];
        if (g->table_h.empty())
            continue;
        PPCG_TRY(ensure_table(*g));
        if (g == &gs_) {
            small_iters = chunk_iters(gs_, kSmallChunkIters);
        } else {
            bool covers = false;
            for (int len : chunk_plan(*g, graph_iters, &covers)) {
                hipGraphExec_t e = nullptr;
                PPCG_TRY(ensure_graph(*g, len, &e));
                execs[k].push_back(e);
            }
            if (covers && !g->pcg)
                finals.push_back(g);
        }
    }
    PPCG_TRY(flush_uploads());
    int nactive = 0;
    for (int k = 0; k < kGroups; ++k)
        nactive += !groups[k]->table_h.empty();
    // with one active group there is nothing to overlap: stay on stream_
    const bool fork = nactive > 1;
    if (fork)
        PPCG_HIP(hipEventRecord(ev_fork_, stream_));
    for (int k = 0; k < kGroups; ++k) {
        Group *g = groups[k];
        if (g->table_h.empty())
            continue;
        hipStream_t gs = fork ? gstream_[k] : stream_;
        if (fork)
            PPCG_HIP(hipStreamWaitEvent(gs, ev_fork_, 0));
        if (g == &gs_) {
            k_small_iter<<<(int)gs_.table_h.size(), kSmallThreads, 0, gs>>>(gs_.table_d, gs_.count_d, gs_.desc_d,
                                                                          small_iters);
            PPCG_HIP(hipGetLastError());
        } else {
            for (hipGraphExec_t e : execs[k])
                PPCG_HIP(hipGraphLaunch(e, gs));
        }
        if (fork) {
            PPCG_HIP(hipEventRecord(ev_join_[k], gs));
            PPCG_HIP(hipStreamWaitEvent(stream_, ev_join_[k], 0));
        }
    }
    // Fixed-iteration jobs whose last iteration was just launched: their
    // true residual follows at once (no poll in between).
    for (Group *g : finals) {
        std::vector<int> slots;
        for (Job &j : jobs_)
            if (!j.finished && j.stage == JS_ITER && &pgroup(j) == g) {
                slots.push_back(pslot(j));
                j.expect_done = true;
            }
        PPCG_TRY(aux_launch(*g, slots, AUX_RESID));
    }
    if (!finals.empty() && after_fixed_final)
        PPCG_TRY(after_fixed_final());
    // 5. Poll the groups that iterated.
    for (Group *g : groups)
        if (!g->table_h.empty())
            PPCG_TRY(sync_states(*g));
    PPCG_HIP(hipStreamSynchronize(stream_));
    for (Job &j : jobs_) {
        if (j.finished || j.stage != JS_ITER)
            continue;
        const Group &g = pgroup(j);
        const SysState &st = g.st_h[pslot(j)];
        const SysDesc &d = g.desc_h[pslot(j)];
        if (j.expect_done) {
            j.expect_done = false;
            if (!st.done) {
                set_error("a fixed-iteration system did not stop after its last launch");
                return PPCG_ERR_DEVICE;
            }
            const double bn = std::sqrt(st.bnorm2);
            j.rel_true = bn > 0 ? std::sqrt(st.tnorm2) / bn : std::sqrt(st.tnorm2);
            const FinalAction act = final_action(j.h->opt, st, j.restarts, j.rel_true, j.tol);
            finish(j, act == FINAL_STAGNATED ? PPCG_STAGNATED : st.status, st);
            continue;
        }
        if (st.done) {
            j.last_norm = -1.0;
            j.rate = -1.0;
            if (j.mixed == MIX_INNER32) {
                j.inner_iters = st.iter;  // the sequence's counter runs across reliable updates
                j.precond_norm = std::sqrt(st.uu);
                j.stage = JS_OUTER;
            } else if (st.status == ST_REPLACE) {
                j.stage = JS_NEED_REPL;
            } else {
                j.stage = JS_NEED_FINAL;
            }
        } else {
            note_progress(d, st, &j.last_norm, &j.last_iter, &j.rate);
        }
    }
    return PPCG_OK;
}

// Iterations per graph chunk: aim for about 4 ms of device work, so that the
// host's poll between chunks costs about 1% of the time.
int auto_graph_iters(const ppcg_handle *h)
{
    if (h->opt.graph_iters > 0)
        return h->opt.graph_iters;
    const ByteModel bm = byte_model(h, PREC_F64);
    const double us = (bm.vma + bm.spmv) / 5.0e6 + 6.0;  // ~5 TB/s plus launch overheads
    int k = (int)(4000.0 / us);
    return std::max(8, std::min(k, 128));
}

// Copy b and x0 into the handle's internal (stored-row order) vectors.
ppcg_status stage_inputs(ppcg_handle *h, const double *b, const double *x0)
{
    h->x0_zero = x0 == nullptr;
    hipStream_t s = h->stream;
    const int n = h->n;
    double *bi = (double *)h->f64.vec[VB], *xi = (double *)h->f64.vec[VX], *tmp = (double *)h->f64.vec[VN];
    const unsigned g = blocks_for(n, 256);
    if (h->opt.vec_mem == PPCG_MEM_HOST) {
        PPCG_HIP(hipMemcpyAsync(tmp, b, sizeof(double) * n, hipMemcpyHostToDevice, s));
        k_gather<double, double><<<g, 256, 0, s>>>(n, h->perm, tmp, bi);
        if (x0) {
            PPCG_HIP(hipMemcpyAsync(tmp, x0, sizeof(double) * n, hipMemcpyHostToDevice, s));
            k_gather<double, double><<<g, 256, 0, s>>>(n, h->perm, tmp, xi);
        }
    } else {
        k_gather<double, double><<<g, 256, 0, s>>>(n, h->perm, b, bi);
        if (x0)
            k_gather<double, double><<<g, 256, 0, s>>>(n, h->perm, x0, xi);
    }
    if (!x0)
        k_fill<double><<<g, 256, 0, s>>>((size_t)n, xi, 0.0);
    PPCG_HIP(hipGetLastError());
    return PPCG_OK;
}

ppcg_status unstage_x(ppcg_handle *h, double *x)
{
    hipStream_t s = h->stream;
    const int n = h->n;
    const double *xi = (const double *)h->f64.vec[VX];
    double *tmp = (double *)h->f64.vec[VN];
    const unsigned g = blocks_for(n, 256);
    if (h->opt.vec_mem == PPCG_MEM_HOST) {
        k_scatter<<<g, 256, 0, s>>>(n, h->perm, xi, tmp);
        PPCG_HIP(hipMemcpyAsync(x, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    } else {
        k_scatter<<<g, 256, 0, s>>>(n, h->perm, xi, x);
    }
    PPCG_HIP(hipGetLastError());
    return PPCG_OK;
}

void fill_info(const ppcg_handle *h, const Job &j, ppcg_info *info)
{
    if (!info)
        return;
    const size_t sz = info->struct_size == sizeof(ppcg_info) ? sizeof(ppcg_info) : 0;
    if (!sz)
        return;
    memset(info, 0, sizeof *info);
    info->struct_size = sizeof *info;
    info->status = (ppcg_status)j.status;
    info->iters = j.iters;
    info->outer_iters = j.outer;
    info->restarts = j.restarts;
    info->rel_resid_true = j.rel_true;
    info->rel_resid_recur = j.rel_recur;
    info->precond_norm = j.precond_norm;
    info->time_ms = j.t_end - j.t_start;
    const ByteModel bm = byte_model(h, j.mixed == MIX_INNER32 ? PREC_F32 : j.mixed == MIX_VALUES32 ? PREC_V32 : PREC_F64);
    info->model_bytes = (bm.vma + bm.spmv) * j.iters;
    info->precision = h->opt.precision;
    info->method = j.pcg ? PPCG_METHOD_PCG : PPCG_METHOD_PIPECG;
}

// Order the internal stream after all work already queued on the caller's
// stream (the legacy default stream when the caller passed NULL).
ppcg_status wait_user(ppcg_handle *h)
{
    PPCG_HIP(hipEventRecord(h->ev_user, h->user_stream));
    PPCG_HIP(hipStreamWaitEvent(h->stream, h->ev_user, 0));
    return PPCG_OK;
}

// The moves of a batch's staging, all systems in one launch.
static ppcg_status launch_stage(hipStream_t s, const BatchCtx &c, const StageItem *items_h, int off, int nitems,
                                int64_t rows)
{
    if (nitems == 0)
        return PPCG_OK;
    PPCG_HIP(hipMemcpyAsync(c.items_d + off, items_h, sizeof(StageItem) * nitems, hipMemcpyHostToDevice, s));
    // about 4 rows per thread on an average item; long items loop
    const int64_t avg = rows / nitems;
    const unsigned gx = (unsigned)std::min<int64_t>(std::max<int64_t>((avg + 1023) / 1024, 1), 256);
    const unsigned gy = (unsigned)std::min(nitems, 65535);
    k_stage_batch<<<dim3(gx, gy), 256, 0, s>>>(c.items_d + off, nitems);
    PPCG_HIP(hipGetLastError());
    return PPCG_OK;
}

// One batched solve on the cached engine: inputs staged (device vectors in
// one launch, host vectors per system), all systems iterated together,
// solutions copied out the same way.
ppcg_status batch_run(BatchCtx &c, int count, ppcg_handle *const *hs, const double *const *b,
                      const double *const *x0, double *const *x, ppcg_info *infos)
{
    hipStream_t s = hs[0]->stream;
    Engine &E = *c.E;
    E.reset();
    // The previous batch on this context ended with a synchronisation, so
    // the pinned table is free.  Regions: [0, 2 cap) inputs, [2 cap, 3 cap) outputs.
    StageItem *in = c.items_h, *out = c.items_h + 2 * (size_t)c.cap;
    int nin = 0, nout = 0;
    int64_t rin = 0, rout = 0;
    for (int i = 0; i < count; ++i) {
        ppcg_handle *h = hs[i];
        const double *xi0 = x0 ? x0[i] : nullptr;
        if (h->opt.vec_mem == PPCG_MEM_HOST) {
            hipStream_t keep = h->stream;
            h->stream = s;
            ppcg_status rc = stage_inputs(h, b[i], xi0);
            h->stream = keep;
            PPCG_TRY(rc);
            continue;
        }
        h->x0_zero = xi0 == nullptr;
        double *bi = (double *)h->f64.vec[VB], *xi = (double *)h->f64.vec[VX];
        in[nin++] = StageItem{h->perm, b[i], bi, h->n, STAGE_GATHER};
        in[nin++] = xi0 ? StageItem{h->perm, xi0, xi, h->n, STAGE_GATHER} : StageItem{nullptr, nullptr, xi, h->n, STAGE_ZERO};
        rin += 2 * (int64_t)h->n;
    }
    PPCG_TRY(launch_stage(s, c, in, 0, nin, rin));
    int gi = 128;
    for (int i = 0; i < count; ++i) {
        int id;
        const int mixed = hs[i]->opt.precision == PPCG_MIXED_FP32 ? MIX_INNER32 : hs[i]->opt.precision == PPCG_MIXED_FP32_VALUES ? MIX_VALUES32 : MIX_NONE;
        PPCG_TRY(E.add(hs[i], mixed, hs[i]->opt.tol, nullptr, &id));
        gi = std::min(gi, auto_graph_iters(hs[i]));
    }
    PPCG_TRY(run_engine(E, std::max(gi, 16)));
    for (int i = 0; i < count; ++i) {
        ppcg_handle *h = hs[i];
        if (h->opt.vec_mem == PPCG_MEM_HOST) {
            hipStream_t keep = h->stream;
            h->stream = s;
            ppcg_status rc = unstage_x(h, x[i]);
            h->stream = keep;
            PPCG_TRY(rc);
            continue;
        }
        out[nout++] = StageItem{h->perm, (const double *)h->f64.vec[VX], x[i], h->n, STAGE_SCATTER};
        rout += h->n;
    }
    PPCG_TRY(launch_stage(s, c, out, 2 * c.cap, nout, rout));
    PPCG_HIP(hipStreamSynchronize(s));
    if (infos)
        for (int i = 0; i < count; ++i)
            fill_info(hs[i], E.job(i), &infos[i]);
    return PPCG_OK;
}

ppcg_status run_engine(Engine &E, int graph_iters)
{
    int guard = 0;
    while (!E.all_done()) {
        PPCG_TRY(E.step(graph_iters));
        if (++guard > 10000000) {
            set_error("engine made no progress");
            return PPCG_ERR_DEVICE;
        }
    }
    return PPCG_OK;
}

ppcg_status check_options(const ppcg_options *o)
{
    if (!o || o->struct_size != sizeof(ppcg_options)) {
        set_error("options NULL or struct_size mismatch");
        return PPCG_ERR_INVALID_ARG;
    }
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol) || o->max_iter < 0 || o->fixed_iters < 0 ||
        o->max_restarts < 0 || o->graph_iters < 0 || o->graph_iters > 4096 || !(o->inner_tol >= 0.0) ||
        o->inner_tol >= 1.0 || o->max_outer < 0 ||
        (o->stop != PPCG_STOP_REL_RESID && o->stop != PPCG_STOP_PRECOND_ABS) ||
        (o->precision != PPCG_FP64 && o->precision != PPCG_MIXED_FP32 && o->precision != PPCG_MIXED_FP32_VALUES) ||
        (o->vec_mem != PPCG_MEM_DEVICE && o->vec_mem != PPCG_MEM_HOST) ||
        (o->spmv_format != PPCG_SPMV_AUTO && o->spmv_format != PPCG_SPMV_SELL &&
         o->spmv_format != PPCG_SPMV_CSR_VECTOR) ||
        (o->method != PPCG_METHOD_PIPECG && o->method != PPCG_METHOD_PCG) ||
        (o->flags & ~(PPCG_FLAG_BORROW_INPUTS | PPCG_FLAG_SELL_COL16 | PPCG_FLAG_SELL_COL32 |
                      PPCG_FLAG_SELL_VALUE_TABLE | PPCG_FLAG_SELL_FULL_VALUES | PPCG_FLAG_ITER_FUSED |
                      PPCG_FLAG_ITER_TWO_LAUNCH | PPCG_FLAG_SELL_SHARED_OFFSETS |
                      PPCG_FLAG_SELL_NO_SHARED_OFFSETS)) != 0 ||
        ((o->flags & PPCG_FLAG_ITER_FUSED) && (o->flags & PPCG_FLAG_ITER_TWO_LAUNCH)) ||
        ((o->flags & PPCG_FLAG_SELL_SHARED_OFFSETS) && (o->flags & PPCG_FLAG_SELL_NO_SHARED_OFFSETS)) ||
        ((o->flags & PPCG_FLAG_SELL_COL16) && (o->flags & PPCG_FLAG_SELL_COL32)) ||
        ((o->flags & PPCG_FLAG_SELL_VALUE_TABLE) && (o->flags & PPCG_FLAG_SELL_FULL_VALUES))) {
        set_error("invalid option value");
        return PPCG_ERR_INVALID_ARG;
    }
    return PPCG_OK;
}

}  // namespace ppcg

using namespace ppcg;

// ======================================================================= ABI

extern "C" {

const char *ppcg_last_error(void) { return g_err.c_str(); }

const char *ppcg_status_str(ppcg_status s)
{
    switch (s) {
    case PPCG_OK: return "PPCG_OK";
    case PPCG_NOT_CONVERGED: return "PPCG_NOT_CONVERGED";
    case PPCG_BREAKDOWN: return "PPCG_BREAKDOWN";
    case PPCG_STAGNATED: return "PPCG_STAGNATED";
    case PPCG_ERR_INVALID_ARG: return "PPCG_ERR_INVALID_ARG";
    case PPCG_ERR_BAD_CSR: return "PPCG_ERR_BAD_CSR";
    case PPCG_ERR_NOMEM: return "PPCG_ERR_NOMEM";
    case PPCG_ERR_DEVICE: return "PPCG_ERR_DEVICE";
    case PPCG_ERR_BUDGET: return "PPCG_ERR_BUDGET";
    }
    return "PPCG_UNKNOWN";
}

ppcg_status ppcg_default_options(ppcg_options *opt)
{
    if (!opt) {
        set_error("opt is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    memset(opt, 0, sizeof *opt);
    opt->struct_size = sizeof *opt;
    opt->tol = 1e-8;
    opt->max_iter = 10000;
    opt->fixed_iters = 0;
    opt->max_restarts = 3;
    opt->stop = PPCG_STOP_REL_RESID;
    opt->precision = PPCG_FP64;
    opt->vec_mem = PPCG_MEM_DEVICE;
    opt->spmv_format = PPCG_SPMV_AUTO;
    opt->graph_iters = 0;
    opt->inner_tol = 0.0;
    opt->max_outer = 30;
    opt->method = PPCG_METHOD_PIPECG;
    opt->flags = 0;
    return PPCG_OK;
}


static void destroy_handle(ppcg_handle *h)
{
    if (!h)
        return;
    if (h->stream)
        (void)hipStreamSynchronize(h->stream);
    delete h->solo;
    h->solo = nullptr;
    delete h->batch;
    h->batch = nullptr;
    plain_free(h);
    free_matrix(h);
    if (h->dinv64)
        (void)dev_free(h->dinv64);
    h->f64.arena.release();
    h->f32.arena.release();
    h->fused_arena.release();
    if (h->ev_user)
        (void)hipEventDestroy(h->ev_user);
    if (h->stream)
        (void)hipStreamDestroy(h->stream);
    delete h;
}

ppcg_status ppcg_create(const ppcg_csr *A, const ppcg_options *opt, void *hip_stream, ppcg_handle **out)
{
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!A || A->struct_size != sizeof(ppcg_csr)) {
        set_error("A NULL or struct_size mismatch");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_TRY(check_options(opt));
    if (A->n < 1 || A->nnz < A->n || A->nnz >= (int64_t)INT_MAX || !A->row_ptr || !A->col_idx || !A->values ||
        (A->mem != PPCG_MEM_DEVICE && A->mem != PPCG_MEM_HOST)) {
        set_error("invalid CSR description (n=%d nnz=%lld)", A->n, (long long)A->nnz);
        return PPCG_ERR_INVALID_ARG;
    }
    const double t0 = now_ms();
    ppcg_handle *h = new ppcg_handle();
    h->opt = *opt;
    h->n = A->n;
    h->nnz = A->nnz;
    h->ntiles = (A->n + kTileRows - 1) / kTileRows;
    h->user_stream = (hipStream_t)hip_stream;
    int *rp = nullptr, *ci = nullptr, *rowlen = nullptr;
    double *val = nullptr, *dinv_orig = nullptr;
    unsigned *err = nullptr;
    bool own_csr = false;
    auto fail = [&](ppcg_status s) {
        if (own_csr) {
            if (rp) (void)dev_free(rp);
            if (ci) (void)dev_free(ci);
            if (val) (void)dev_free(val);
        }
        if (rowlen) (void)dev_free(rowlen);
        if (dinv_orig) (void)dev_free(dinv_orig);
        if (err) (void)dev_free(err);
        destroy_handle(h);
        return s;
    };
#define CK(call)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            set_error("%s failed: %s", #call, hipGetErrorString(e_));                         \
            return fail(e_ == hipErrorOutOfMemory ? PPCG_ERR_NOMEM : PPCG_ERR_DEVICE);        \
        }                                                                                     \
    } while (0)
#define CKS(expr)                   \
    do {                            \
        ppcg_status s_ = (expr);    \
        if (s_ != PPCG_OK)          \
            return fail(s_);        \
    } while (0)
    CK(hipGetDevice(&h->device));
    CK(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device));
    CK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    CK(hipEventCreateWithFlags(&h->ev_user, hipEventDisableTiming));
    hipStream_t s = h->stream;
    CK(hipEventRecord(h->ev_user, h->user_stream));
    CK(hipStreamWaitEvent(s, h->ev_user, 0));
    const int n = A->n;
    const int64_t nnz = A->nnz;
    if (A->mem == PPCG_MEM_HOST) {
        own_csr = true;
        CK(hipMalloc(&rp, sizeof(int) * (n + 1)));
        CK(hipMalloc(&ci, sizeof(int) * nnz));
        CK(hipMalloc(&val, sizeof(double) * nnz));
        CK(hipMemcpyAsync(rp, A->row_ptr, sizeof(int) * (n + 1), hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(ci, A->col_idx, sizeof(int) * nnz, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(val, A->values, sizeof(double) * nnz, hipMemcpyHostToDevice, s));
    } else {
        CKS(check_dev_range(A->row_ptr, sizeof(int) * (n + 1), "row_ptr"));
        CKS(check_dev_range(A->col_idx, sizeof(int) * nnz, "col_idx"));
        CKS(check_dev_range(A->values, sizeof(double) * nnz, "values"));
        rp = (int *)A->row_ptr;
        ci = (int *)A->col_idx;
        val = (double *)A->values;
    }
    CK(hipMalloc(&rowlen, sizeof(int) * n));
    CK(hipMalloc(&dinv_orig, sizeof(double) * n));
    CK(hipMalloc(&h->dinv64, sizeof(double) * n));
    CK(hipMalloc(&err, sizeof(unsigned) * 2));
    unsigned err_init[2] = {0u, 0xFFFFFFFFu};
    CK(hipMemcpyAsync(err, err_init, sizeof err_init, hipMemcpyHostToDevice, s));
    k_validate<<<blocks_for(n, 256), 256, 0, s>>>(n, nnz, rp, ci, val, dinv_orig, rowlen, err);
    CK(hipGetLastError());
    unsigned err_h[2];
    CK(hipMemcpyAsync(err_h, err, sizeof err_h, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (err_h[0]) {
        set_csr_error(err_h);
        return fail(PPCG_ERR_BAD_CSR);
    }
    std::vector<int> rowlen_h(n);
    // on the handle's stream: a copy on the null stream synchronizes with the
    // device and would invalidate a graph capture under way in another thread
    CK(hipMemcpyAsync(rowlen_h.data(), rowlen, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    {
        // A constant diagonal makes M^-1 a multiple of the identity: the fused
        // updates then read dinv[0] for every row (one cached line) instead
        // of streaming the dinv vector.
        unsigned zero = 0u, differs = 1u;
        CK(hipMemcpyAsync(err, &zero, sizeof zero, hipMemcpyHostToDevice, s));
        k_const_check<<<blocks_for(n, 256), 256, 0, s>>>(n, dinv_orig, err);
        CK(hipGetLastError());
        CK(hipMemcpyAsync(&differs, err, sizeof differs, hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        h->dinv_const = differs == 0u;
    }
    CKS(alloc_f64_vectors(h));
    CKS(choose_format(h, rp, ci, val, rowlen, dinv_orig, rowlen_h));
    CKS(tune_vtab(h, A->mem == PPCG_MEM_HOST ? A->values : nullptr, val));
    CKS(tune_shared(h));
    CKS(tune_form(h));
    shared_for_fused(h);
    if (opt->precision == PPCG_MIXED_FP32)
        CKS(ensure_f32(h));
    if (opt->precision == PPCG_MIXED_FP32_VALUES)
        CKS(ensure_val32(h));
    CK(hipStreamSynchronize(s));
    if (own_csr) {
        (void)dev_free(rp);
        (void)dev_free(ci);
        (void)dev_free(val);
    }
    (void)dev_free(rowlen);
    (void)dev_free(dinv_orig);
    (void)dev_free(err);
    h->setup_ms = now_ms() - t0;
    *out = h;
    return PPCG_OK;
#undef CK
#undef CKS
}

ppcg_status ppcg_set_options(ppcg_handle *h, const ppcg_options *opt)
{
    clear_error();
    if (!h) {
        set_error("handle is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_TRY(check_options(opt));
    if (opt->spmv_format != h->opt.spmv_format && opt->spmv_format != PPCG_SPMV_AUTO) {
        set_error("the SpMV format is fixed at creation");
        return PPCG_ERR_INVALID_ARG;
    }
    ppcg_spmv_format keep = h->opt.spmv_format;
    h->opt = *opt;
    h->opt.spmv_format = keep;
    if (opt->precision == PPCG_MIXED_FP32)
        PPCG_TRY(ensure_f32(h));
    if (opt->precision == PPCG_MIXED_FP32_VALUES)
        PPCG_TRY(ensure_val32(h));
    return PPCG_OK;
}

ppcg_status ppcg_destroy(ppcg_handle *h)
{
    clear_error();
    destroy_handle(h);
    return PPCG_OK;
}

static ppcg_status check_vec(const ppcg_handle *h, const void *p, const char *what, bool may_null)
{
    if (!p) {
        if (may_null)
            return PPCG_OK;
        set_error("%s is NULL", what);
        return PPCG_ERR_INVALID_ARG;
    }
    if (h->opt.vec_mem == PPCG_MEM_DEVICE)
        return check_dev_range(p, sizeof(double) * (size_t)h->n, what);
    return PPCG_OK;
}

ppcg_status ppcg_solve(ppcg_handle *h, const double *b, const double *x0, double *x, ppcg_info *info)
{
    clear_error();
    if (!h) {
        set_error("handle is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    if (info && info->struct_size != sizeof(ppcg_info)) {
        set_error("info struct_size mismatch");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_TRY(check_vec(h, b, "b", false));
    PPCG_TRY(check_vec(h, x0, "x0", true));
    PPCG_TRY(check_vec(h, x, "x", false));
    PPCG_HIP(hipSetDevice(h->device));
    PPCG_TRY(wait_user(h));
    PPCG_TRY(stage_inputs(h, b, x0));
    if (!h->solo) {
        h->solo = new Engine(h->stream);
        PPCG_TRY(h->solo->init(1));
    }
    Engine &E = *h->solo;
    E.reset();  // the solo engine is reused: one job per solve
    int id = -1;
    const int mixed = h->opt.precision == PPCG_MIXED_FP32 ? MIX_INNER32 : h->opt.precision == PPCG_MIXED_FP32_VALUES ? MIX_VALUES32 : MIX_NONE;
    PPCG_TRY(E.add(h, mixed, h->opt.tol, nullptr, &id));
    // a fixed-iteration solve copies x out behind its true residual, before
    // the engine's last poll; otherwise after the engine has finished
    bool unstaged = false;
    E.after_fixed_final = [&]() -> ppcg_status {
        unstaged = true;
        return unstage_x(h, x);
    };
    ppcg_status rc = run_engine(E, auto_graph_iters(h));
    E.after_fixed_final = nullptr;
    PPCG_TRY(rc);
    if (!unstaged)
        PPCG_TRY(unstage_x(h, x));
    PPCG_HIP(hipStreamSynchronize(h->stream));
    Job &j = E.job(id);
    j.t_end = now_ms();
    fill_info(h, j, info);
    return (ppcg_status)j.status;
}

ppcg_status ppcg_solve_batch(int32_t count, ppcg_handle *const *hs, const double *const *b, const double *const *x0,
                             double *const *x, ppcg_info *infos)
{
    clear_error();
    if (count < 1 || !hs || !b || !x) {
        set_error("invalid batch arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    for (int i = 0; i < count; ++i) {
        if (!hs[i]) {
            set_error("hs[%d] is NULL", i);
            return PPCG_ERR_INVALID_ARG;
        }
        for (int k = 0; k < i; ++k)
            if (hs[k] == hs[i]) {
                set_error("handle %d appears twice in the batch", i);
                return PPCG_ERR_INVALID_ARG;
            }
        if (hs[i]->device != hs[0]->device) {
            set_error("handles on different devices");
            return PPCG_ERR_INVALID_ARG;
        }
        if (infos && infos[i].struct_size != sizeof(ppcg_info)) {
            set_error("infos[%d] struct_size mismatch", i);
            return PPCG_ERR_INVALID_ARG;
        }
        PPCG_TRY(check_vec(hs[i], b[i], "b[i]", false));
        PPCG_TRY(check_vec(hs[i], x0 ? x0[i] : nullptr, "x0[i]", true));
        PPCG_TRY(check_vec(hs[i], x[i], "x[i]", false));
    }
    ppcg_handle *h0 = hs[0];
    PPCG_HIP(hipSetDevice(h0->device));
    hipStream_t s = h0->stream;
    // b[i] and x0[i] may come from work queued on any handle's stream: the
    // batch waits for every distinct one before it stages the inputs.
    {
        std::vector<hipStream_t> seen;
        for (int i = 0; i < count; ++i) {
            if (std::find(seen.begin(), seen.end(), hs[i]->user_stream) != seen.end())
                continue;
            seen.push_back(hs[i]->user_stream);
            hipStream_t keep = hs[i]->stream;
            hs[i]->stream = s;
            ppcg_status rc = wait_user(hs[i]);
            hs[i]->stream = keep;
            PPCG_TRY(rc);
        }
    }
    // The first handle keeps the batch's engine and staging table for the
    // next batch it leads (of at most as many systems).
    if (!h0->batch || h0->batch->cap < count) {
        delete h0->batch;
        h0->batch = new BatchCtx;
        BatchCtx &c = *h0->batch;
        c.E = new Engine(s);
        PPCG_TRY(c.E->init(count));
        PPCG_HIP(hipMalloc(&c.items_d, sizeof(StageItem) * 3 * (size_t)count));
        PPCG_HIP(hipHostMalloc((void **)&c.items_h, sizeof(StageItem) * 3 * (size_t)count, hipHostMallocDefault));
        c.cap = count;  // usable only once complete
    }
    ppcg_status rc = batch_run(*h0->batch, count, hs, b, x0, x, infos);
    if (rc < 0) {
        // start the next batch from a fresh engine
        delete h0->batch;
        h0->batch = nullptr;
    }
    return rc;
}

ppcg_status ppcg_get_matrix_info(const ppcg_handle *h, ppcg_matrix_info *mi)
{
    clear_error();
    if (!h || !mi || mi->struct_size != sizeof(ppcg_matrix_info)) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    memset(mi, 0, sizeof *mi);
    mi->struct_size = sizeof *mi;
    mi->n = h->n;
    mi->nnz = h->nnz;
    mi->nnz_stored = h->nnz_stored;
    mi->format = (ppcg_spmv_format)h->fmt;
    mi->sell_c = kSellC;
    mi->sell_sigma = h->sigma;
    mi->lanes_per_row = h->lanes;
    mi->tile_rows = kTileRows;
    const ByteModel bm = byte_model(h, h->opt.precision == PPCG_MIXED_FP32 ? PREC_F32
                                       : h->opt.precision == PPCG_MIXED_FP32_VALUES ? PREC_V32 : PREC_F64);
    mi->bytes_vma = bm.vma;
    mi->bytes_spmv = bm.spmv;
    mi->bytes_per_iter = bm.vma + bm.spmv;
    mi->device_bytes = (double)h->f64.arena.size + (double)h->f32.arena.size +
                       (double)h->nnz_stored * 12.0 + 8.0 * h->n +
                       (h->fmt == FMT_SELL ? 8.0 * (h->nchunks + 1) : 4.0 * (h->n + 1)) +
                       (h->perm ? 8.0 * h->n : 0.0) + (h->col16 ? 2.0 * (double)h->nnz_stored : 0.0) +
                       (h->vidx ? (double)h->nnz_stored + 8.0 * h->nvtab : 0.0) +
                       (h->cpat ? 4.0 * (h->nchunks + h->npats) : 0.0);
    mi->setup_ms = h->setup_ms;
    mi->col_index_bytes =
        h->shared_on ? 0
        : (h->col16 && (PPCG_PCG_V32_COL16 ||
                        !(h->opt.method == PPCG_METHOD_PCG && h->opt.precision == PPCG_MIXED_FP32_VALUES))) ? 2
                                                                                                             : 4;
    mi->diag_const = h->dinv_const ? 1 : 0;
    const bool pcg = h->opt.method == PPCG_METHOD_PCG || h->opt.precision == PPCG_MIXED_FP32;
    mi->value_bytes = h->opt.precision == PPCG_MIXED_FP32 || h->opt.precision == PPCG_MIXED_FP32_VALUES ? 4
                      : (h->vidx && !pcg)                                                              ? 1
                                                                                                       : 8;
    mi->distinct_values = h->nvtab;
    mi->iter_launches = (h->form == FORM_FUSED && !pcg && h->opt.precision == PPCG_FP64) ? 1 : 2;
    return PPCG_OK;
}

double ppcg_footprint_bytes(int32_t n, int64_t nnz, ppcg_precision precision)
{
    if (n < 1 || nnz < n)
        return 0.0;
    const double ntiles = (n + kTileRows - 1) / kTileRows;
    const double stored = 1.10 * (double)nnz;  // padding allowance
    // stored entries: 8 value + 4 column + 2 (16-bit column offsets, when
    // built) + 1 (value index, when built) bytes
    double b = stored * 15.0 + 8.0 * (n / kSellC + 2) + 8.0 * n /* dinv */ + 8.0 * n /* perm */ +
               11.0 * 8.0 * n + 2.0 * ntiles * kPartStride * 8.0 + 12 * 256.0;
    if (precision == PPCG_MIXED_FP32)
        b += stored * 4.0 + 12.0 * 4.0 * n + 2.0 * ntiles * kPartStride * 8.0;
    if (precision == PPCG_MIXED_FP32_VALUES)
        b += stored * 4.0;
    return b;
}

ppcg_status ppcg_time_kernels(ppcg_handle *h, const double *b, int32_t iters, double *ms_vma, double *ms_spmv)
{
    clear_error();
    if (!h || iters < 1 || iters > 100000 || !ms_vma || !ms_spmv) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_TRY(check_vec(h, b, "b", false));
    PPCG_HIP(hipSetDevice(h->device));
    PPCG_TRY(wait_user(h));
    PPCG_TRY(stage_inputs(h, b, nullptr));
    hipStream_t s = h->stream;
    // Fixed-iteration mode with a count larger than iters: never stops early.
    PPCG_TRY(plain_setup(h, 0.0, INT_MAX, INT_MAX));
    std::vector<hipEvent_t> ev(4 * iters, nullptr);
    auto clean = [&]() {
        (void)hipStreamSynchronize(s);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    const int grid = h->ntiles;
    const WorkItem *tab = h->plain_tab;
    const int *cnt = h->plain_cnt;
    const SysDesc *dd = h->plain_desc;
    const bool pcg = h->opt.method == PPCG_METHOD_PCG;
    if (!pcg && h->form == FORM_FUSED) {
        // the single-launch form: its one kernel, after the initialisation
        // and the launch that ends it
        const int fgrid = fused_tiles(h);
        launch_pipecg_init_fused(s, tab, cnt, dd, grid);
        k_fused_begin<<<fgrid, 64, 0, s>>>(tab, cnt + 1, dd);
        k_fused<<<fgrid, kFusedThreads, 0, s>>>(tab, cnt + 1, dd, PPCG_FUSED_REMAP, 0);
        for (auto &e : ev)
            PPCG_HIP_CLEAN(hipEventCreate(&e), clean());
        for (int i = 1; i <= iters; ++i)
            hipExtLaunchKernelGGL(k_fused, dim3(fgrid), dim3(kFusedThreads), 0, s, ev[4 * (i - 1)],
                                  ev[4 * (i - 1) + 1], 0, tab, cnt + 1, dd, (int)PPCG_FUSED_REMAP, i & 1);
        PPCG_HIP_CLEAN(hipGetLastError(), clean());
        PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
        double tf = 0;
        for (int i = 0; i < iters; ++i) {
            float a = 0;
            PPCG_HIP_CLEAN(hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]), clean());
            tf += a;
        }
        *ms_vma = tf / iters;
        *ms_spmv = 0.0;
        clean();
        return PPCG_OK;
    }
    k_spmv<double, MODE_INIT1><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, PPCG_XCD_REMAP_SPMV);
    if (pcg) {
        k_pcg_dots<double><<<grid, kVmaThreads, 0, s>>>(tab, cnt, dd);
        k_pcg_update<PCG_START><<<1, kPcgRedThreads, 0, s>>>(tab, cnt, dd);  // item 0 is (system, tile 0)
    } else {
        k_spmv<double, MODE_INIT2><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, PPCG_XCD_REMAP_SPMV);
        k_spmv<double, MODE_ITER><<<grid, kSpmvThreads, 0, s>>>(tab, cnt, dd, PPCG_XCD_REMAP_SPMV);
    }
    for (auto &e : ev)
        PPCG_HIP_CLEAN(hipEventCreate(&e), clean());
    // Events attached to each launch (start/stop of the kernel itself), so
    // the durations exclude the gaps between launches.
    for (int i = 0; i < iters; ++i) {
        const int rv = (int)PPCG_XCD_REMAP, rs = (int)PPCG_XCD_REMAP_SPMV;
        if (pcg) {
            // the two streaming kernels are timed; the per-system reductions
            // between them run untimed
            hipExtLaunchKernelGGL(k_pcg_spmv<double>, dim3(grid), dim3(kSpmvThreads), 0, s, ev[4 * i + 2], ev[4 * i + 3], 0,
                                  tab, cnt, dd, rs);
            k_pcg_alpha<<<1, kPcgRedThreads, 0, s>>>(tab, cnt, dd);
            hipExtLaunchKernelGGL(k_pcg_vma<double>, dim3(grid), dim3(kVmaThreads), 0, s, ev[4 * i], ev[4 * i + 1], 0, tab,
                                  cnt, dd, rv);
            k_pcg_update<PCG_ITER><<<1, kPcgRedThreads, 0, s>>>(tab, cnt, dd);
        } else {
            hipExtLaunchKernelGGL(k_vma<double>, dim3(grid), dim3(kVmaThreads), 0, s, ev[4 * i], ev[4 * i + 1], 0,
                                  tab, cnt, dd, rv);
            hipExtLaunchKernelGGL((k_spmv<double, MODE_ITER>), dim3(grid), dim3(kSpmvThreads), 0, s,
                                  ev[4 * i + 2], ev[4 * i + 3], 0, tab, cnt, dd, rs);
        }
    }
    PPCG_HIP_CLEAN(hipGetLastError(), clean());
    PPCG_HIP_CLEAN(hipStreamSynchronize(s), clean());
    double tv = 0, ts = 0;
    for (int i = 0; i < iters; ++i) {
        float a = 0, c = 0;
        PPCG_HIP_CLEAN(hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]), clean());
        PPCG_HIP_CLEAN(hipEventElapsedTime(&c, ev[4 * i + 2], ev[4 * i + 3]), clean());
        tv += a;
        ts += c;
    }
    *ms_vma = tv / iters;
    *ms_spmv = ts / iters;
    clean();
    return PPCG_OK;
}

ppcg_status ppcg_spmv(ppcg_handle *h, const double *x, double *y)
{
    clear_error();
    if (!h) {
        set_error("handle is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_TRY(check_vec(h, x, "x", false));
    PPCG_TRY(check_vec(h, y, "y", false));
    if (x == y) {
        set_error("x and y must not alias");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_HIP(hipSetDevice(h->device));
    PPCG_TRY(wait_user(h));
    // stage x into the internal x vector (stored-row order)
    PPCG_TRY(stage_inputs(h, x, x));
    PPCG_TRY(plain_setup(h, 1e-8, 0, 1));
    hipStream_t s = h->stream;
    k_spmv<double, MODE_PLAIN><<<h->ntiles, kSpmvThreads, 0, s>>>(h->plain_tab, h->plain_cnt, h->plain_desc, PPCG_XCD_REMAP_SPMV);
    PPCG_HIP(hipGetLastError());
    // result is in the internal nv vector; scatter it out like x
    const int n = h->n;
    const unsigned g = blocks_for(n, 256);
    double *nv = (double *)h->f64.vec[VN], *tmp = (double *)h->f64.vec[VZ];
    if (h->opt.vec_mem == PPCG_MEM_HOST) {
        k_scatter<<<g, 256, 0, s>>>(n, h->perm, nv, tmp);
        PPCG_HIP(hipMemcpyAsync(y, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    } else {
        k_scatter<<<g, 256, 0, s>>>(n, h->perm, nv, y);
    }
    PPCG_HIP(hipStreamSynchronize(s));
    return PPCG_OK;
}

}  // extern "C"
