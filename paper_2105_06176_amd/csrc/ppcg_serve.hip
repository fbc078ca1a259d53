// ppcg_serve.hip -- continuous-batching solve server (ppcg_srv_* in ppcg.h).
//
// Requests queue on the host.  Preparation threads owned by the server take
// them first-come first-served while the sum of the device footprints of the
// requests the server holds (in preparation, prepared, or on the device)
// stays within the budget, and prepare each one on a stream of its own: the
// matrix is copied to the device, validated and laid out (ppcg_create) and
// the right-hand side staged.  Each scheduling step admits the prepared
// requests, in the order they became ready, into the shared batched engine,
// runs one graph chunk of PIPECG iterations over every active request, and
// retires the requests that finished: a preparation thread copies their
// solutions back to the host and releases their device memory.  Preparation
// and release
// therefore overlap with the iterations of the requests already on the
// device (releasing memory synchronizes the device), and requests that arrive
// while others iterate join the batched launches at the next chunk
// boundary.  A request's arithmetic is independent of the mix: it owns its
// tiles, partial sums and scalars.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ppcg_engine.hpp"

using namespace ppcg;

namespace {

constexpr int kServerSlots = 1024;
// iterations per graph chunk (a power of two): requests finish, and new ones
// join, at chunk boundaries
#ifndef PPCG_SERVE_GRAPH_ITERS
#define PPCG_SERVE_GRAPH_ITERS 8
#endif
constexpr int kServeGraphIters = PPCG_SERVE_GRAPH_ITERS;
// preparation threads: requests are prepared concurrently (copy, validation,
// layout and staging), taken first come first served, admitted as they
// become ready
#ifndef PPCG_SERVE_PREP_THREADS
#define PPCG_SERVE_PREP_THREADS 2
#endif
constexpr int kPrepThreads = PPCG_SERVE_PREP_THREADS;
// automatic precision: smallest systems given reduced precision
#ifndef PPCG_AUTO_VALUES32_ROWS
#define PPCG_AUTO_VALUES32_ROWS 65536
#endif
#ifndef PPCG_AUTO_PCG32_ROWS
#define PPCG_AUTO_PCG32_ROWS 262144
#endif
constexpr int kAutoValues32Rows = PPCG_AUTO_VALUES32_ROWS;
constexpr int kAutoPcg32Rows = PPCG_AUTO_PCG32_ROWS;

enum ReqState { RQ_QUEUED, RQ_PREPARING, RQ_PREPARED, RQ_ACTIVE, RQ_FINISHING, RQ_DONE };

struct Request {
    int64_t id = 0;
    ReqState state = RQ_QUEUED;
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
};

}  // namespace

// Ownership: the preparation thread that took a request alone touches it in
// state RQ_PREPARING or RQ_FINISHING; the calling thread alone touches one in
// RQ_PREPARED or RQ_ACTIVE.  The map, the queues, the counters and every
// state change are guarded by `mu`.
struct ppcg_server {
    hipStream_t stream = nullptr;       // the engine's stream
    hipStream_t prep_stream = nullptr;  // orders each preparation (its handle has a stream of its own)
    int device = 0;
    ppcg_options defaults{};
    double budget = 0.0;
    int64_t next_id = 1;
    std::unique_ptr<Engine> eng;
    std::mutex mu;
    std::condition_variable prep_cv;   // wakes the preparation threads
    std::condition_variable ready_cv;  // wakes a step that waits for a prepared request
    std::map<int64_t, Request> reqs;
    std::deque<int64_t> queue;  // awaiting preparation, first come first served
    std::deque<int64_t> ready;  // prepared, awaiting admission, in the order they became ready
    // Retired requests: a preparation thread copies the solution out and
    // releases the handle (a release synchronizes the device), then marks
    // the request ready to poll, or queues it again for an FP64 rerun.
    struct Retired {
        int64_t id;
        ppcg_handle *h;
        double footprint;
        bool rerun;
    };
    std::vector<Retired> retired;
    int finishing = 0;          // retired requests not yet ready to poll
    double used = 0.0;          // footprints of the handles in preparation, prepared, active or retired
    int preparing = 0;
    int active = 0;
    bool stop = false;
    ppcg_status prep_rc = PPCG_OK;  // a device error met while preparing, reported by the next step
    std::string prep_msg;
    std::vector<std::thread> prep;
};

// A preparation thread may take the first queued request: within the slot
// count, and within the budget unless nothing else holds device memory (a
// retired request holds its memory until it is released).
static bool can_prepare(const ppcg_server *s)
{
    if (s->stop || s->prep_rc != PPCG_OK || s->queue.empty())
        return false;
    const int held = s->active + (int)s->ready.size() + s->preparing;
    if (held >= kServerSlots)
        return false;
    const Request &r = s->reqs.at(s->queue.front());
    return (held == 0 && s->finishing == 0) || s->used + r.footprint <= s->budget;
}

// Copy the request's matrix and right-hand side to the device (runs on a
// preparation thread, unlocked).  A request whose matrix ppcg_create refuses
// fails on its own; a device error is returned.
static ppcg_status prepare(ppcg_server *s, Request &r)
{
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
    ppcg_status rc = ppcg_create(&A, &o, s->prep_stream, &r.h);
    if (rc != PPCG_OK) {
        r.h = nullptr;
        memset(&r.info, 0, sizeof r.info);
        r.info.struct_size = sizeof r.info;
        r.info.status = rc;
        return PPCG_OK;
    }
    // a rerun (automatic precision fallback) starts from the last iterate
    rc = stage_inputs(r.h, r.b_p, r.x.empty() ? nullptr : r.x.data());
    if (rc == PPCG_OK && hipStreamSynchronize(r.h->stream) != hipSuccess) {
        set_error("staging the right-hand side failed");
        rc = PPCG_ERR_DEVICE;
    }
    if (rc != PPCG_OK) {
        ppcg_destroy(r.h);
        r.h = nullptr;
    }
    return rc;
}

static void prep_loop(ppcg_server *s)
{
    const bool dev_ok = hipSetDevice(s->device) == hipSuccess;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!dev_ok) {
        s->prep_rc = PPCG_ERR_DEVICE;
        s->prep_msg = "hipSetDevice failed on a preparation thread";
        s->ready_cv.notify_all();
        return;
    }
    for (;;) {
        s->prep_cv.wait(lk, [s] { return s->stop || !s->retired.empty() || can_prepare(s); });
        if (!s->retired.empty()) {
            std::vector<ppcg_server::Retired> batch;
            batch.swap(s->retired);
            std::vector<Request *> rs;
            for (auto &e : batch)
                rs.push_back(&s->reqs.at(e.id));
            lk.unlock();
            ppcg_status rc = PPCG_OK;
            for (size_t k = 0; k < batch.size(); ++k) {
                Request &r = *rs[k];
                if (rc == PPCG_OK) {
                    r.x.assign(r.n, 0.0);
                    rc = unstage_x(batch[k].h, r.x.data());
                    if (rc == PPCG_OK && hipStreamSynchronize(batch[k].h->stream) != hipSuccess) {
                        set_error("copying the solution out failed");
                        rc = PPCG_ERR_DEVICE;
                    }
                }
                ppcg_destroy(batch[k].h);
            }
            std::string msg = rc == PPCG_OK ? std::string() : std::string(ppcg_last_error());
            lk.lock();
            for (size_t k = 0; k < batch.size(); ++k) {
                Request &r = *rs[k];
                s->used -= batch[k].footprint;
                --s->finishing;
                if (batch[k].rerun && rc == PPCG_OK) {
                    // reduced precision did not reach the tolerance: run again
                    // in FP64 from the last iterate, ahead of the requests not
                    // yet prepared
                    r.state = RQ_QUEUED;
                    s->queue.push_front(batch[k].id);
                    continue;
                }
                r.state = RQ_DONE;
                if (rc != PPCG_OK)
                    r.info.status = rc;
                std::vector<double>().swap(r.b);
                std::vector<int32_t>().swap(r.rp);
                std::vector<int32_t>().swap(r.ci);
                std::vector<double>().swap(r.val);
            }
            if (rc != PPCG_OK) {
                s->prep_rc = rc;
                s->prep_msg = msg;
            }
            s->ready_cv.notify_all();
            s->prep_cv.notify_all();  // memory released: another thread may prepare
            continue;
        }
        if (s->stop)
            return;
        const int64_t id = s->queue.front();
        s->queue.pop_front();
        Request &r = s->reqs.at(id);  // map nodes stay put while others come and go
        r.state = RQ_PREPARING;
        s->used += r.footprint;
        ++s->preparing;
        lk.unlock();
        const ppcg_status rc = prepare(s, r);
        std::string msg = rc == PPCG_OK ? std::string() : std::string(ppcg_last_error());
        lk.lock();
        --s->preparing;
        if (r.h) {
            r.state = RQ_PREPARED;
            s->ready.push_back(id);
        } else {
            s->used -= r.footprint;
            r.state = RQ_DONE;
            if (rc != PPCG_OK) {
                r.info.struct_size = sizeof r.info;
                r.info.status = rc;
                s->prep_rc = rc;
                s->prep_msg = msg;
            }
        }
        s->ready_cv.notify_all();
    }
}

// Admit the prepared requests (calling thread, under `mu`).
static ppcg_status admit(ppcg_server *s)
{
    while (!s->ready.empty()) {
        Request &r = s->reqs.at(s->ready.front());
        s->ready.pop_front();
        const int mixed = r.precision == PPCG_MIXED_FP32          ? MIX_INNER32
                          : r.precision == PPCG_MIXED_FP32_VALUES ? MIX_VALUES32
                                                                  : MIX_NONE;
        ppcg_status rc = s->eng->add(r.h, mixed, r.tol, nullptr, &r.job);
        if (rc != PPCG_OK) {
            ppcg_destroy(r.h);
            r.h = nullptr;
            s->used -= r.footprint;
            r.state = RQ_DONE;
            memset(&r.info, 0, sizeof r.info);
            r.info.struct_size = sizeof r.info;
            r.info.status = rc;
            s->prep_cv.notify_one();
            return rc;
        }
        r.state = RQ_ACTIVE;
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

// Retire the requests whose job finished (calling thread, under `mu`); the
// preparation thread copies their solutions out.
static ppcg_status retire_finished(ppcg_server *s)
{
    for (auto &kv : s->reqs) {
        Request &r = kv.second;
        if (r.state != RQ_ACTIVE)
            continue;
        Job &j = s->eng->job(r.job);
        if (!j.finished)
            continue;
        r.info.struct_size = sizeof r.info;
        fill_info(r.h, j, &r.info);
        s->eng->retire(r.job);
        const bool budget_spent =
            r.info.status == PPCG_NOT_CONVERGED && r.info.outer_iters >= s->defaults.max_outer;
        const bool rerun = r.auto_prec && r.precision != PPCG_FP64 &&
                           (r.info.status == PPCG_STAGNATED || r.info.status == PPCG_BREAKDOWN || budget_spent);
        // the memory counts until it is released
        s->retired.push_back({kv.first, r.h, r.footprint, rerun});
        r.h = nullptr;
        r.state = RQ_FINISHING;
        --s->active;
        ++s->finishing;
        if (rerun) {
            r.precision = PPCG_FP64;
            r.method = s->defaults.method;
            r.footprint = ppcg_footprint_bytes(r.n, r.nnz, PPCG_FP64);
        }
    }
    if (!s->retired.empty()) {
        // the engine's last chunk must be complete before another stream reads x
        PPCG_HIP(hipStreamSynchronize(s->eng->stream()));
        s->prep_cv.notify_one();
    }
    return PPCG_OK;
}

static ppcg_status take_prep_error(ppcg_server *s)
{
    if (s->prep_rc == PPCG_OK)
        return PPCG_OK;
    set_error("request preparation: %s", s->prep_msg.c_str());
    return s->prep_rc;
}

extern "C" {

ppcg_status ppcg_srv_create(const ppcg_options *opt, double budget_bytes, ppcg_server **out)
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
    PPCG_HIP(hipGetDevice(&s->device));
    PPCG_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->eng.reset(new Engine(s->stream));
    ppcg_status rc = s->eng->init(kServerSlots);
    if (rc == PPCG_OK && hipStreamCreateWithFlags(&s->prep_stream, hipStreamNonBlocking) != hipSuccess) {
        set_error("creating the preparation stream failed");
        rc = PPCG_ERR_DEVICE;
    }
    if (rc == PPCG_OK) {
        try {
            for (int t = 0; t < kPrepThreads; ++t)
                s->prep.emplace_back(prep_loop, s.get());
        } catch (...) {
            set_error("starting the preparation thread failed");
            rc = PPCG_ERR_NOMEM;
        }
    }
    if (rc != PPCG_OK) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->prep_cv.notify_all();
        for (std::thread &t : s->prep)
            t.join();
        s->eng.reset();
        if (s->prep_stream)
            (void)hipStreamDestroy(s->prep_stream);
        (void)hipStreamDestroy(s->stream);
        return rc;
    }
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
    std::unique_lock<std::mutex> lk(s->mu);
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
    lk.unlock();
    s->prep_cv.notify_one();
    return PPCG_OK;
}

ppcg_status ppcg_srv_step(ppcg_server *s, int32_t *active, int32_t *queued)
{
    clear_error();
    if (!s) {
        set_error("server is NULL");
        return PPCG_ERR_INVALID_ARG;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    PPCG_TRY(take_prep_error(s));
    // with nothing on the device, wait for the next prepared request
    if (s->active == 0)
        s->ready_cv.wait(lk, [s] {
            return !s->ready.empty() || s->prep_rc != PPCG_OK ||
                   (s->preparing == 0 && s->queue.empty() && s->finishing == 0);
        });
    PPCG_TRY(take_prep_error(s));
    PPCG_TRY(admit(s));
    if (s->active > 0) {
        // the engine and the active requests belong to this thread
        lk.unlock();
        PPCG_TRY(s->eng->step(kServeGraphIters));
        lk.lock();
        PPCG_TRY(retire_finished(s));
    }
    if (active)
        *active = s->active + s->finishing;
    if (queued)
        *queued = (int32_t)(s->queue.size() + s->ready.size()) + s->preparing;
    return PPCG_OK;
}

ppcg_status ppcg_srv_poll(ppcg_server *s, int64_t req_id, int32_t *ready, double *x, ppcg_info *info)
{
    clear_error();
    if (!s || !ready) {
        set_error("invalid arguments");
        return PPCG_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) {
        set_error("unknown request id %lld", (long long)req_id);
        return PPCG_ERR_INVALID_ARG;
    }
    Request &r = it->second;
    if (r.state != RQ_DONE) {
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
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->prep_cv.notify_all();
    for (std::thread &t : s->prep)
        t.join();  // a preparation under way completes first
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->reqs)
        if (kv.second.h)
            ppcg_destroy(kv.second.h);
    for (auto &e : s->retired)
        ppcg_destroy(e.h);
    s->eng.reset();
    if (s->prep_stream)
        (void)hipStreamDestroy(s->prep_stream);
    if (s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
    return PPCG_OK;
}

}  // extern "C"
