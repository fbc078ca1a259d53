// ppcg_serve.hip -- continuous-batching solve server (ppcg_srv_* in ppcg.h).
//
// Requests queue on the host.  Each scheduling step admits queued requests
// first-come first-served while the sum of their device footprints stays
// within the budget (and the engine has free slots), then runs one graph
// chunk of PIPECG iterations over every active request through the shared
// batched engine, and retires requests that finished: their solution is
// copied back to the host and their device memory released.  Requests that
// arrive while others are on the device therefore join the batched launches
// at the next chunk boundary and overlap with them.  A request's arithmetic
// is independent of the mix: it owns its tiles, partial sums and scalars.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "ppcg_engine.hpp"

using namespace ppcg;

namespace {

constexpr int kServerSlots = 1024;
constexpr int kServeGraphIters = 32;
// automatic precision: smallest systems given reduced precision
#ifndef PPCG_AUTO_VALUES32_ROWS
#define PPCG_AUTO_VALUES32_ROWS 65536
#endif
#ifndef PPCG_AUTO_PCG32_ROWS
#define PPCG_AUTO_PCG32_ROWS 262144
#endif
constexpr int kAutoValues32Rows = PPCG_AUTO_VALUES32_ROWS;
constexpr int kAutoPcg32Rows = PPCG_AUTO_PCG32_ROWS;

struct Request {
    int64_t id = 0;
    int state = 0;  // 0 queued, 1 active, 2 finished
    double footprint = 0.0;
    double tol = 0.0;
    ppcg_precision precision = PPCG_FP64;
    ppcg_method method = PPCG_METHOD_PIPECG;
    bool auto_prec = false;  // chosen by the server; reduced precision falls back to FP64
    int32_t n = 0;
    int64_t nnz = 0;
    // inputs: owned copies, or the caller's arrays (borrowing server)
    std::vector<int32_t> rp, ci;
    std::vector<double> val, b, x;
    const int32_t *rp_p = nullptr, *ci_p = nullptr;
    const double *val_p = nullptr, *b_p = nullptr;
    ppcg_handle *h = nullptr;
    int job = -1;
    ppcg_info info{};
    ppcg_status create_status = PPCG_OK;
};

}  // namespace

struct ppcg_server {
    hipStream_t stream = nullptr;
    ppcg_options defaults{};
    double budget = 0.0;
    double used = 0.0;
    int64_t next_id = 1;
    std::unique_ptr<Engine> eng;
    std::map<int64_t, Request> reqs;
    std::deque<int64_t> queue;
    int active = 0;
};

static ppcg_status admit(ppcg_server *s)
{
    while (!s->queue.empty() && s->active < kServerSlots) {
        Request &r = s->reqs[s->queue.front()];
        if (s->used + r.footprint > s->budget && s->active > 0)
            break;  // wait for memory to free up (first come, first served)
        s->queue.pop_front();
        ppcg_options o = s->defaults;
        o.tol = r.tol;
        o.precision = r.precision;
        o.method = r.method;
        o.vec_mem = PPCG_MEM_HOST;
        o.fixed_iters = 0;
        ppcg_csr A{};
        A.struct_size = sizeof A;
        A.n = r.n;
        A.nnz = r.nnz;
        A.row_ptr = r.rp_p;
        A.col_idx = r.ci_p;
        A.values = r.val_p;
        A.mem = PPCG_MEM_HOST;
        ppcg_status rc = ppcg_create(&A, &o, s->stream, &r.h);
        if (rc != PPCG_OK) {
            // The request fails on its own; the server keeps going.
            r.state = 2;
            r.create_status = rc;
            memset(&r.info, 0, sizeof r.info);
            r.info.struct_size = sizeof r.info;
            r.info.status = rc;
            continue;
        }
        PPCG_TRY(wait_user(r.h));
        hipStream_t keep = r.h->stream;
        r.h->stream = s->eng->stream();
        // a rerun (automatic precision fallback) starts from the last iterate
        rc = stage_inputs(r.h, r.b_p, r.x.empty() ? nullptr : r.x.data());
        r.h->stream = keep;
        PPCG_TRY(rc);
        const int mixed = r.precision == PPCG_MIXED_FP32          ? MIX_INNER32
                          : r.precision == PPCG_MIXED_FP32_VALUES ? MIX_VALUES32
                                                                  : MIX_NONE;
        PPCG_TRY(s->eng->add(r.h, mixed, r.tol, nullptr, &r.job));
        r.state = 1;
        s->used += r.footprint;
        ++s->active;
        // inputs now live on the device (kept while a fallback rerun may need them)
        if (!(r.auto_prec && r.precision != PPCG_FP64)) {
            std::vector<int32_t>().swap(r.rp);
            std::vector<int32_t>().swap(r.ci);
            std::vector<double>().swap(r.val);
            r.rp_p = r.ci_p = nullptr;
            r.val_p = nullptr;
        }
    }
    return PPCG_OK;
}

static ppcg_status retire_finished(ppcg_server *s)
{
    for (auto &kv : s->reqs) {
        Request &r = kv.second;
        if (r.state != 1)
            continue;
        Job &j = s->eng->job(r.job);
        if (!j.finished)
            continue;
        r.x.assign(r.n, 0.0);
        hipStream_t keep = r.h->stream;
        r.h->stream = s->eng->stream();
        ppcg_status rc = unstage_x(r.h, r.x.data());
        r.h->stream = keep;
        PPCG_TRY(rc);
        PPCG_HIP(hipStreamSynchronize(s->eng->stream()));
        r.info.struct_size = sizeof r.info;
        fill_info(r.h, j, &r.info);
        s->eng->retire(r.job);
        ppcg_destroy(r.h);
        r.h = nullptr;
        s->used -= r.footprint;
        --s->active;
        const bool budget_spent =
            r.info.status == PPCG_NOT_CONVERGED && r.info.outer_iters >= s->defaults.max_outer;
        if (r.auto_prec && r.precision != PPCG_FP64 &&
            (r.info.status == PPCG_STAGNATED || r.info.status == PPCG_BREAKDOWN || budget_spent)) {
            // reduced precision did not reach the tolerance: run again in
            // FP64 from the last iterate, ahead of the requests still queued
            r.precision = PPCG_FP64;
            r.method = s->defaults.method;
            r.footprint = ppcg_footprint_bytes(r.n, r.nnz, PPCG_FP64);
            r.state = 0;
            s->queue.push_front(kv.first);
            continue;
        }
        r.state = 2;
        std::vector<double>().swap(r.b);
        std::vector<int32_t>().swap(r.rp);
        std::vector<int32_t>().swap(r.ci);
        std::vector<double>().swap(r.val);
    }
    return PPCG_OK;
}

extern "C" {

ppcg_status ppcg_srv_create(const ppcg_options *opt, double budget_bytes, void *hip_stream, ppcg_server **out)
{
    clear_error();
    if (!out || !opt || opt->struct_size != sizeof(ppcg_options) || !(budget_bytes >= 0.0)) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    std::unique_ptr<ppcg_server> s(new ppcg_server());
    s->defaults = *opt;
    if (budget_bytes == 0.0) {
        size_t fr = 0, tot = 0;
        PPCG_HIP(hipMemGetInfo(&fr, &tot));
        budget_bytes = 0.8 * (double)fr;
    }
    s->budget = budget_bytes;
    PPCG_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    (void)hip_stream;  // requests are ordered on the server's own stream
    s->eng.reset(new Engine(s->stream));
    PPCG_TRY(s->eng->init(kServerSlots));
    *out = s.release();
    return PPCG_OK;
}

ppcg_status ppcg_srv_submit(ppcg_server *s, const ppcg_csr *A, const double *b, double tol, ppcg_precision precision,
                            int64_t *req_id)
{
    clear_error();
    if (!s || !A || !b || !req_id || A->struct_size != sizeof(ppcg_csr) || A->mem != PPCG_MEM_HOST || A->n < 1 ||
        A->nnz < A->n || !A->row_ptr || !A->col_idx || !A->values || !(tol >= 0.0) ||
        (precision != PPCG_FP64 && precision != PPCG_MIXED_FP32 && precision != PPCG_MIXED_FP32_VALUES &&
         precision != PPCG_PRECISION_AUTO)) {
        set_error("invalid request");
        return PPCG_ERR_INVALID_ARG;
    }
    const bool auto_prec = precision == PPCG_PRECISION_AUTO;
    ppcg_method method = s->defaults.method;
    if (auto_prec) {
        // bytes of one iteration: FP64 PIPECG 12 per stored entry plus 17
        // FP64 vector streams per row; FP32 values 8 per entry; classic PCG
        // in FP32 8 per entry plus 12 FP32 vector streams per row, with two
        // more launches per iteration (one-workgroup reductions), so it is
        // taken only where the bytes saved clearly outweigh them; below
        // 65536 rows launch latency, not bytes, sets the time
        const double b64 = 12.0 * (double)A->nnz + 136.0 * A->n;
        const double bv32 = 8.0 * (double)A->nnz + 136.0 * A->n;
        const double bp32 = 8.0 * (double)A->nnz + 48.0 * A->n;
        if (A->n >= kAutoPcg32Rows && bp32 <= 0.7 * b64) {
            precision = PPCG_MIXED_FP32;  // always Algorithm 1
            method = PPCG_METHOD_PCG;
        } else if (A->n >= kAutoValues32Rows && bv32 <= 0.95 * b64) {
            precision = PPCG_MIXED_FP32_VALUES;
        } else {
            precision = PPCG_FP64;
        }
    }
    const double fp = ppcg_footprint_bytes(A->n, A->nnz, precision);
    if (fp > s->budget) {
        set_error("request footprint %.0f bytes exceeds the budget %.0f", fp, s->budget);
        return PPCG_ERR_BUDGET;
    }
    Request r;
    r.id = s->next_id++;
    r.footprint = fp;
    r.tol = tol;
    r.precision = precision;
    r.method = method;
    r.auto_prec = auto_prec;
    r.n = A->n;
    r.nnz = A->nnz;
    if (s->defaults.flags & PPCG_FLAG_BORROW_INPUTS) {
        r.rp_p = A->row_ptr;
        r.ci_p = A->col_idx;
        r.val_p = A->values;
        r.b_p = b;
    } else {
        r.rp.assign(A->row_ptr, A->row_ptr + A->n + 1);
        r.ci.assign(A->col_idx, A->col_idx + A->nnz);
        r.val.assign(A->values, A->values + A->nnz);
        r.b.assign(b, b + A->n);
        r.rp_p = r.rp.data();
        r.ci_p = r.ci.data();
        r.val_p = r.val.data();
        r.b_p = r.b.data();
    }
    *req_id = r.id;
    s->queue.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
    return PPCG_OK;
}

ppcg_status ppcg_srv_step(ppcg_server *s, int32_t *active, int32_t *queued)
{
    clear_error();
    if (!s) {
        set_error("server is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    PPCG_TRY(admit(s));
    if (s->active > 0) {
        PPCG_TRY(s->eng->step(kServeGraphIters));
        PPCG_TRY(retire_finished(s));
    }
    if (active)
        *active = s->active;
    if (queued)
        *queued = (int32_t)s->queue.size();
    return PPCG_OK;
}

ppcg_status ppcg_srv_poll(ppcg_server *s, int64_t req_id, int32_t *ready, double *x, ppcg_info *info)
{
    clear_error();
    if (!s || !ready) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) {
        set_error("unknown request id %lld", (long long)req_id);
        return PPCG_ERR_INVALID_ARG;
    }
    Request &r = it->second;
    if (r.state != 2) {
        *ready = 0;
        return PPCG_NOT_CONVERGED;
    }
    *ready = 1;
    if (x && !r.x.empty())
        memcpy(x, r.x.data(), sizeof(double) * r.n);
    if (info && info->struct_size == sizeof(ppcg_info))
        *info = r.info;
    const ppcg_status st = r.info.status;
    s->reqs.erase(it);
    return st;
}

ppcg_status ppcg_srv_destroy(ppcg_server *s)
{
    clear_error();
    if (!s)
        return PPCG_OK;
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->reqs)
        if (kv.second.h)
            ppcg_destroy(kv.second.h);
    s->eng.reset();
    if (s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
    return PPCG_OK;
}

}  // extern "C"
