// ppcg_engine.hpp -- host runtime of the PIPECG library: handles, the
// batched iteration engine and the error channel.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <functional>
#include <cstdio>
#include <map>
#include <string>
#include <mutex>
#include <shared_mutex>
#include <vector>

#include "../../include/ppcg.h"
#include "ppcg_internal.hpp"

namespace ppcg {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

#define PPCG_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::ppcg::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                              __FILE__, __LINE__);                                        \
            return e_ == hipErrorOutOfMemory ? PPCG_ERR_NOMEM : PPCG_ERR_DEVICE;          \
        }                                                                                 \
    } while (0)

#define PPCG_TRY(expr)                        \
    do {                                      \
        ppcg_status s_ = (expr);              \
        if (s_ < 0)                           \
            return s_;                        \
    } while (0)

// ---------------------------------------------------------------- releases
// Releasing device or pinned host memory synchronizes the whole device, and
// a device synchronization while another thread captures a graph invalidates
// that capture.  Every release in the library therefore holds this lock
// shared, and a graph capture holds it exclusively.
std::shared_mutex &release_mu();
inline hipError_t dev_free(void *p)
{
    std::shared_lock<std::shared_mutex> lk(release_mu());
    return hipFree(p);
}
inline hipError_t host_free(void *p)
{
    std::shared_lock<std::shared_mutex> lk(release_mu());
    return hipHostFree(p);
}

// ---------------------------------------------------------------- device buffers
// A single device allocation cut into 256-byte aligned pieces.
struct DevArena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    ppcg_status alloc(size_t bytes);
    void *take(size_t bytes);
    void release();
};

// Matrix + vectors of one precision for one handle.
struct PrecData {
    bool ready = false;
    int prec = PREC_F64;
    void *val = nullptr;   // SELL or CSR values in this precision
    void *dinv = nullptr;
    void *vec[11] = {};    // x r u w m nv z q s p b
    DevArena arena;
};

enum VecIdx { VX = 0, VR, VU, VW, VM, VN, VZ, VQ, VS, VP, VB };

// How an FP64 PIPECG iteration is launched: the fused update and the SpMV as
// two launches (ppcg_kernels.hpp), or one launch (ppcg_fused.hpp).
enum IterForm { FORM_TWO = 0, FORM_FUSED = 1 };

class Engine;
struct BatchCtx;
struct StageItem;

}  // namespace ppcg

struct ppcg_handle {
    int device = 0;
    int cus = 0;  // compute units of the device
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;  // internal stream (capturable), ordered after user_stream
    ppcg_options opt{};
    int n = 0;
    int64_t nnz = 0;
    int ntiles = 0;
    // matrix storage (format independent pieces)
    int fmt = ppcg::FMT_SELL;
    int lanes = 0;
    int sigma = 1;
    int nchunks = 0;
    int64_t nnz_stored = 0;
    int64_t *cptr = nullptr;  // SELL chunk offsets
    int *rp = nullptr;        // CSR row pointers (CSR-vector format)
    int *col = nullptr;
    short *col16 = nullptr;   // SELL: 16-bit column offsets from the row, when they all fit
    unsigned char *vidx = nullptr;  // SELL: one-byte index of each stored value in vtab
    double *vtab = nullptr;   // the distinct values (ascending bit patterns) when vidx is set
    int nvtab = 0;
    // SELL, rows in their own order: each chunk's shared offset list (the
    // chunk's entry k of every row at column row + pats[cpat[c] + k]) when
    // every chunk has one; shared_on: the FP64 PIPECG SpMV reads them
    int *cpat = nullptr, *pats = nullptr;
    int npats = 0;
    bool shared_on = false;
    int *perm = nullptr, *invperm = nullptr;
    double *val64 = nullptr;  // FP64 values in the stored format
    float *val32 = nullptr;   // FP32 copy of the stored values (mixed modes)
    double *dinv64 = nullptr;
    bool dinv_const = false;  // every diagonal entry equal (e.g. constant-coefficient stencils)
    ppcg::DevArena mat_arena;
    ppcg::PrecData f64, f32;
    double *part = nullptr;   // 2 x ntiles x 4 partial sums (shared by both precisions)
    double *part32 = nullptr; // partials of the FP32-vector sequence
    double setup_ms = 0.0;
    ppcg::Engine *solo = nullptr;  // cached single-system engine
    ppcg::BatchCtx *batch = nullptr;  // cached engine of batches led by this handle
    hipEvent_t ev_user = nullptr;  // recorded on user_stream for the internal stream to wait on
    // Single-system launch description for direct kernel calls (SpMV,
    // kernel timing, autotuning): descriptor, state, table of all tiles.
    ppcg::SysDesc *plain_desc = nullptr;
    ppcg::SysState *plain_st = nullptr;
    ppcg::WorkItem *plain_tab = nullptr;
    int *plain_cnt = nullptr;
    // Iteration form of FP64 PIPECG (IterForm): two launches per iteration or
    // the single-launch form, chosen at create time; the single-launch form's
    // buffers (state and partial-sum slots, second w buffer).
    int form = 0;
    bool x0_zero = false;  // the last staged initial guess was zero (no x0 given)
    ppcg::SysState *frec = nullptr;
    double *fpart = nullptr;
    double *w1 = nullptr;
    ppcg::DevArena fused_arena;
};

namespace ppcg {

// One solve in progress inside an engine.
struct Job {
    ppcg_handle *h = nullptr;
    int mixed = 0;          // 0 FP64, 1 FP32 inner PIPECG + FP64 refinement,
                            // 2 FP32 values + reliable updates (MixKind)
    int slot64 = -1;        // slot in the FP64 group (MIX_NONE, and the outer FP64 steps of MIX_INNER32)
    int slot32 = -1;        // slot in the FP32-vector classic-PCG group (MIX_INNER32)
    int slotv = -1;         // slot in the FP32-values group (MIX_VALUES32)
    int stage = 0;          // JobStage
    int restarts = 0;
    int outer = 0;
    int inner_iters = 0;
    int status = PPCG_OK;
    double tol = 0.0;
    bool finished = false;
    double t_start = 0.0, t_end = 0.0;
    double rel_true = 0.0, rel_recur = 0.0, precond_norm = 0.0;
    double bnorm2 = 0.0;
    int iters = 0;
    // convergence tracking for choosing graph chunk lengths: the stopping
    // quantity and iteration count at the last poll of the current start
    // (last_norm < 0: not polled yet), and the mean reduction factor per
    // iteration between the last two polls (< 0: unknown)
    double last_norm = -1.0;
    int last_iter = 0;
    double rate = -1.0;
    // MIX_VALUES32: residual norm right after the last replacement (-1: unknown)
    double repl_ref = -1.0;
    // FP64 system small enough for the one-workgroup iteration kernel
    bool small = false;
    // classic PCG (Algorithm 1) instead of PIPECG
    bool pcg = false;
    // FP64 PIPECG in the single-launch form
    bool fused = false;
    // the initialisation has run once (a later one is a restart from x)
    bool started = false;
    // the initial guess is zero: the first initialisation needs no SpMV
    bool x0_zero = false;
    // fixed-iteration job whose remaining iterations were all launched in
    // this step, with its true residual enqueued behind them
    bool expect_done = false;
};

enum MixKind { MIX_NONE = 0, MIX_INNER32 = 1, MIX_VALUES32 = 2 };

enum JobStage {
    JS_NEED_INIT = 0,   // FP64 group: run the initialisation, then iterate
    JS_ITER = 1,        // iterating in the group's table
    JS_NEED_FINAL = 2,  // FP64 group: true residual, then restart / replace or finish
    JS_OUTER = 3,       // MIX_INNER32: true residual of x, then finish, or start / continue the FP32 sequence
    JS_NEED_REPL = 4,   // MIX_VALUES32: residual replacement (reliable update)
    JS_DONE = 5
};

// Per-precision set of system slots, work table and captured graph.
struct Group {
    int prec = PREC_F64;
    bool pcg = false;               // iterates Algorithm 1 (two launches per iteration, PAR alternating)
    bool fused = false;             // FP64 PIPECG, one launch per iteration (work items are fused tiles)
    int cap_sys = 0;
    SysDesc *desc_d = nullptr;
    SysState *st_d = nullptr;
    SysState *st_h = nullptr;       // pinned mirror
    std::vector<SysDesc> desc_h;
    std::vector<char> slot_used;
    WorkItem *table_d = nullptr;
    int *count_d = nullptr;
    int table_cap = 0;
    WorkItem *aux_d = nullptr;
    int *aux_count_d = nullptr;
    int aux_cap = 0;
    std::vector<WorkItem> aux_h;    // items last uploaded to aux_d (an unchanged table is not re-sent)
    std::vector<SysDesc> desc_up;   // descriptors last uploaded to desc_d
    // Uploads and state clears requested since the last flush (sent as one
    // copy / clear per run of consecutive slots)
    std::vector<char> desc_pending, st_pending;
    SysDesc *desc_stage_h = nullptr;  // pinned staging of descriptor uploads
    WorkItem *stage_h = nullptr;    // pinned staging for table uploads
    int *stage_cnt_h = nullptr;
    int stage_cap = 0;
    std::vector<WorkItem> table_h;  // current iteration table
    std::vector<WorkItem> table_up; // the table last uploaded to table_d (and sys_d)
    bool table_dirty = true;
    // classic PCG groups: one item (slot, 0) per iterating system, for the
    // per-system reduction kernels
    WorkItem *sys_d = nullptr;
    int *sys_count_d = nullptr;
    int sys_cap = 0;
    int nsys = 0;
    int g_sys_grid = 0;
    // Captured graphs of K iterations (K a power of two), all for grid g_grid.
    struct CapturedGraph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<int, CapturedGraph> graphs;
    int g_grid = 0;
};

class Engine {
  public:
    explicit Engine(hipStream_t stream) : stream_(stream) {}
    ~Engine();
    ppcg_status init(int cap_sys);
    // Add a job; returns its index.
    ppcg_status add(ppcg_handle *h, int mixed, double tol, const double *b_dev_internal, int *job_id);
    // Advance all jobs by one scheduling step (transitions + one graph chunk).
    ppcg_status step(int graph_iters);
    bool all_done() const;
    int active() const;
    Job &job(int i) { return jobs_[i]; }
    int njobs() const { return (int)jobs_.size(); }
    // Release a job's slots (serving); the job entry stays for its results.
    void retire(int job_id);
    // Release every job and forget them.
    void reset();
    hipStream_t stream() const { return stream_; }
    int remap = PPCG_XCD_REMAP;
    // Work to enqueue on the engine's stream right behind the true residual
    // of fixed-iteration jobs whose last iteration was launched in the same
    // step (a solo solve copies x out there, saving a host round trip); it
    // runs for such jobs only, and before the step's poll.
    std::function<ppcg_status()> after_fixed_final;

  private:
    ppcg_status ensure_group(Group &g, int prec, int cap_sys);
    // Queue the upload of a slot's descriptor (skipped when unchanged) and
    // the clearing of its state; flush_uploads() sends what is queued, in
    // one copy and one clear per run of consecutive slots, ahead of any
    // launch that reads them.
    ppcg_status upload_desc(Group &g, int slot);
    void clear_state(Group &g, int slot) { g.st_pending[slot] = 1; }
    ppcg_status flush_uploads();
    // `inner`: the group of the FP32 sequences (AUX_MIX_START, AUX_MIX_CORRECT)
    ppcg_status aux_launch(Group &g, const std::vector<int> &slots, int what, const Group *inner = nullptr);
    ppcg_status ensure_table(Group &g);
    ppcg_status ensure_graph(Group &g, int iters, hipGraphExec_t *exec);
    void drop_graphs(Group &g);
    int chunk_iters(const Group &g, int max_iters);
    // Graph lengths to launch back to back for group g before the next
    // poll: one chunk, or, when every iterating job of the group runs a
    // fixed number of iterations, as many chunks as cover them (at most
    // kFixedChunksPerPoll): such jobs need no poll to decide how long to run.
    // *covers: the chunks run every fixed-iteration job of the group to its end.
    std::vector<int> chunk_plan(const Group &g, int max_iters, bool *covers);
    // group and slot where a job iterates
    Group &pgroup(const Job &j)
    {
        if (j.mixed == MIX_INNER32)
            return gp32_;
        if (j.pcg)
            return j.mixed == MIX_VALUES32 ? gpv_ : gp_;
        return j.mixed == MIX_VALUES32 ? gv_ : j.small ? gs_ : j.fused ? gf_ : g64_;
    }
    int pslot(const Job &j) const { return j.mixed == MIX_INNER32 ? j.slot32 : j.mixed == MIX_VALUES32 ? j.slotv : j.slot64; }
    ppcg_status sync_states(Group &g);
    int alloc_slot(Group &g);
    hipStream_t stream_;
    // Each group iterates on a stream of its own (forked from stream_ after
    // the tables and auxiliary work, joined back before the poll), so the
    // groups' launches overlap: the one-workgroup small-system kernel and the
    // graphs of groups holding systems of different precision or method.
    static constexpr int kGroups = 7;
    hipStream_t gstream_[kGroups] = {};
    hipEvent_t ev_fork_ = nullptr;
    hipEvent_t ev_desc_ = nullptr;  // the last flush's descriptor copies (staging reuse)
    bool desc_copy_queued_ = false;
    hipEvent_t ev_join_[kGroups] = {};
    Group g64_, gv_, gs_;   // FP64 (and the FP64 steps of FP32-vector jobs), FP32 values, small systems
    Group gf_;              // FP64 PIPECG in the single-launch form
    Group gp_, gpv_, gp32_; // classic PCG: FP64, FP32 values, FP32 vectors
    std::vector<Job> jobs_;
};

// What ppcg_solve_batch keeps on the batch's first handle between calls:
// the engine (its buffers, streams and captured graphs serve the next batch
// of at most `cap` systems led by the same handle) and the item table of
// the batched staging kernel (inputs in, solutions out).
struct BatchCtx {
    Engine *E = nullptr;
    int cap = 0;
    StageItem *items_d = nullptr;  // 3 x cap items: two per system in, one out
    StageItem *items_h = nullptr;  // pinned staging of the same
    ~BatchCtx();
};

// What follows a stopped FP64 sequence (Algorithm 2, or 1 with FP64 values)
// once its true residual rel = ||b - A x|| / ||b|| is known: restart from x
// when the recurrence met a relative tolerance the true residual misses, or
// after a breakdown past the first iteration of a start (the recurrences
// lost near the attainable accuracy), while restarts and iterations remain;
// a missed tolerance with no restart left is STAGNATED; anything else ends
// with the sequence's own status.
enum FinalAction { FINAL_DONE = 0, FINAL_RESTART = 1, FINAL_STAGNATED = 2 };
inline FinalAction final_action(const ppcg_options &o, const SysState &st, int restarts, double rel, double tol)
{
    const bool tol_mode = o.fixed_iters <= 0;
    const bool can_restart = tol_mode && restarts < o.max_restarts && st.iter < o.max_iter;
    if (st.status == ST_OK && tol_mode && o.stop == PPCG_STOP_REL_RESID && rel > tol)
        return can_restart ? FINAL_RESTART : FINAL_STAGNATED;
    if (st.status == ST_BREAKDOWN && st.i_start > 0 && can_restart)
        return FINAL_RESTART;
    return FINAL_DONE;
}

// Aux operations run over a subset of slots.
// AUX_START: the first initialisation of a job (x holds the staged initial
// guess, nothing deferred); AUX_INIT: a restart from the current x.
// AUX_START0: a first start from x0 = 0 (r0 = b without a pass over A).
enum AuxOp {
    AUX_INIT = 0,
    AUX_RESID = 1,
    AUX_MIX_START = 2,
    AUX_MIX_CORRECT = 3,
    AUX_REPL = 4,
    AUX_START = 5,
    AUX_START0 = 6
};

// Graph chunks a step may launch back to back for fixed-iteration jobs.
constexpr int kFixedChunksPerPoll = 16;

// Launch sequences of FP64 Algorithm 2 over a work table (grid = table
// size), shared by the engine and ppcg_solve_noalloc:
//   launch_x_complete   add the deferred x-update, if any, then clear it;
//   launch_pipecg_init  the initialisation: r0 = b - A x, u0, w0, m0, n0 and
//                       the reduction that yields the first alpha and beta;
//   launch_pipecg_iter  one iteration (fused update, SpMV with reduction);
//   launch_true_resid   ||b - A x||^2 and ||b||^2 into the state record.
void launch_x_complete(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid);
void launch_pipecg_init(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid,
                        bool x_zero = false);
void launch_pipecg_iter(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid, int remap);
// The initialisation of the single-launch form: r0, u0, w0, m0 and the
// partials of the first dot products (its first launch computes n0 and the
// first alpha and beta itself).
void launch_pipecg_init_fused(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid,
                              bool x_zero = false);
// K launches of the single-launch form over a table of fused tiles (K even),
// preceded by k_fused_begin.
void launch_fused_chunk(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid, int iters);
// Allocate the single-launch form's buffers of a handle (once).
ppcg_status ensure_fused(ppcg_handle *h);
// Fused tiles of a handle's system (fused_tile_rows(n, cus) rows each).
int fused_tiles(const ppcg_handle *h);
void launch_true_resid(hipStream_t s, const WorkItem *tab, const int *cnt, const SysDesc *dd, int grid);
// CSR validation (ppcg_create's checks): dinv = 1 / diag, rowlen, and in
// err[0] the OR of the error flags, err[1] the first offending row (err must
// hold {0, 0xFFFFFFFF} before the launch); set_csr_error names the flags.
void launch_validate(hipStream_t s, int n, int64_t nnz, const int *rp, const int *ci, const double *val,
                     double *dinv, int *rowlen, unsigned *err);
void set_csr_error(const unsigned (&err)[2]);
ppcg_status check_options(const ppcg_options *o);
int csrv_default_lanes(double mean_row_length);

// Iterations a running system still needs: exact in fixed-iteration mode,
// else predicted from st (the last poll) and the reduction factor per
// iteration observed between the last two polls (rate < 0: unknown, then
// max_iters); polled: st belongs to the current start.  At least 1, at most
// max_iters.
int iters_needed(const SysDesc &d, const SysState &st, double rate, bool polled, int max_iters, bool pcg);
// After a poll of a running system: update the reduction factor per
// iteration since the previous poll, and remember this poll's norm and count.
void note_progress(const SysDesc &d, const SysState &st, double *last_norm, int *last_iter, double *rate);
double now_ms();
// NULL, non-device and too-short device buffers are rejected with a message.
ppcg_status check_dev_range(const void *p, size_t bytes, const char *what);
int auto_graph_iters(const ppcg_handle *h);
// Helpers shared by the solver API and the server.
ppcg_status stage_inputs(ppcg_handle *h, const double *b, const double *x0);
ppcg_status unstage_x(ppcg_handle *h, double *x);
void fill_info(const ppcg_handle *h, const Job &j, ppcg_info *info);
ppcg_status wait_user(ppcg_handle *h);
ppcg_status run_engine(Engine &E, int graph_iters);
ppcg_status fill_desc(ppcg_handle *h, int prec, SysState *st, SysDesc *d, double tol, int fixed, int maxit,
                      int stop, int vals32 = 0);
ppcg_status ensure_f32(ppcg_handle *h);
ppcg_status ensure_val32(ppcg_handle *h);

}  // namespace ppcg
