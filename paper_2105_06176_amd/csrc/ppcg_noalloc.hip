// ppcg_noalloc.hip -- ppcg_solve_noalloc: Algorithm 2 (PIPECG, FP64, Jacobi)
// on a CSR matrix already in device memory, with every buffer the kernels
// need beyond the caller's inputs and output taken from one statically
// allocated device array, so that the call allocates nothing.
//
// It runs the same kernels, in the same order and on the same tiles, as
// ppcg_solve on a handle created with the CSR-vector format (lanes per row
// as csrv_default_lanes gives them): the initialisation, one fused update +
// SpMV pair per iteration, the true residual, and restarts from x as
// final_action decides.  Results are therefore bitwise equal to that solve.
// Iterations are launched directly (no graph) in chunks whose length follows
// the engine's prediction, and the state record is read back after each
// chunk into host stack memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "ppcg_engine.hpp"

namespace ppcg {
namespace {

// Largest system: 2^19 rows (1,024 tiles).  Layout of the scratch array:
// nine solver vectors (r u w m n z q s p) and the inverse diagonal of
// kNaMaxRows doubles each, the partial sums (2 slots x tiles x 8 doubles),
// the work table, the descriptor, the state record, the tile count and the
// validation flags.  The CSR row lengths that validation writes alias the n
// vector (unused until the first iteration).
constexpr int kNaMaxRows = 1 << 19;
constexpr int kNaMaxTiles = kNaMaxRows / kTileRows;
constexpr size_t kNaVec = (size_t)kNaMaxRows * sizeof(double);
constexpr size_t kNaOffVec = 0;                                     // 10 vectors
constexpr size_t kNaOffPart = kNaOffVec + 10 * kNaVec;
constexpr size_t kNaPartBytes = (size_t)2 * kNaMaxTiles * kPartStride * sizeof(double);
constexpr size_t kNaOffTable = kNaOffPart + kNaPartBytes;
constexpr size_t kNaOffDesc = kNaOffTable + (size_t)kNaMaxTiles * sizeof(WorkItem);
constexpr size_t kNaOffState = kNaOffDesc + ((sizeof(SysDesc) + 255) / 256) * 256;
constexpr size_t kNaOffCount = kNaOffState + 256;
constexpr size_t kNaOffErr = kNaOffCount + 256;
constexpr size_t kNaScratchBytes = kNaOffErr + 256;
static_assert(kNaOffPart % 256 == 0 && kNaOffTable % 256 == 0 && kNaOffDesc % 256 == 0, "aligned pieces");
static_assert(sizeof(SysState) <= 256, "state fits its piece");

constexpr int kNaMaxDevices = 64;

// Iterations per chunk between two reads of the state record (at most).
constexpr int kNaMaxChunk = 64;

// The fills the call needs (work table, tile count, validation flags, a
// zeroed state record), by a kernel rather than hipMemsetAsync.
__global__ void k_na_setup(int ntiles, WorkItem *__restrict__ table, int *__restrict__ count,
                           unsigned *__restrict__ err, double *__restrict__ st)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles)
        table[t] = WorkItem{0, t};
    if (t == 0) {
        *count = ntiles;
        err[0] = 0u;
        err[1] = 0xFFFFFFFFu;
    }
    if (t < (int)(sizeof(SysState) / sizeof(double)))
        st[t] = 0.0;
}

__global__ void k_na_zero(int n, double *__restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        x[i] = 0.0;
}

}  // namespace

// The scratch array itself.  Each device the library runs on holds its own
// copy (about 40 MiB) until the process ends.  In host code its name is only
// a stand-in: host code uses the device address that hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

namespace {

std::mutex g_na_mu[kNaMaxDevices];   // one call per device at a time
unsigned char *g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on device dev, looked up once per device
// (caller holds g_na_mu[dev] and has dev current).
ppcg_status na_scratch(int dev, unsigned char **out)
{
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return PPCG_ERR_DEVICE;
        }
        g_na_ptr[dev] = (unsigned char *)p;
    }
    *out = g_na_ptr[dev];
    return PPCG_OK;
}

ppcg_status na_read_state(hipStream_t s, const SysState *st_d, SysState *st_h)
{
    PPCG_HIP(hipMemcpyAsync(st_h, st_d, sizeof(SysState), hipMemcpyDeviceToHost, s));
    PPCG_HIP(hipStreamSynchronize(s));
    return PPCG_OK;
}

ppcg_status na_solve(const ppcg_csr *A, const ppcg_options *o, const double *b, const double *x0, double *x,
                     ppcg_info *info, hipStream_t s, unsigned char *base)
{
    const double t0 = now_ms();
    const int n = A->n;
    const int64_t nnz = A->nnz;
    const int ntiles = (n + kTileRows - 1) / kTileRows;
    double *vec[10];
    for (int k = 0; k < 10; ++k)
        vec[k] = (double *)(base + kNaOffVec + k * kNaVec);
    double *part = (double *)(base + kNaOffPart);
    WorkItem *table = (WorkItem *)(base + kNaOffTable);
    SysDesc *desc = (SysDesc *)(base + kNaOffDesc);
    SysState *st = (SysState *)(base + kNaOffState);
    int *count = (int *)(base + kNaOffCount);
    unsigned *err = (unsigned *)(base + kNaOffErr);
    double *dinv = vec[9];
    int *rowlen = (int *)vec[4];  // the n vector

    k_na_setup<<<(ntiles + 255) / 256, 256, 0, s>>>(ntiles, table, count, err, (double *)st);
    launch_validate(s, n, nnz, A->row_ptr, A->col_idx, A->values, dinv, rowlen, err);
    PPCG_HIP(hipGetLastError());
    unsigned err_h[2] = {0u, 0u};
    PPCG_HIP(hipMemcpyAsync(err_h, err, sizeof err_h, hipMemcpyDeviceToHost, s));
    PPCG_HIP(hipStreamSynchronize(s));
    if (err_h[0]) {
        set_csr_error(err_h);
        return PPCG_ERR_BAD_CSR;
    }

    const int stop = o->stop == PPCG_STOP_PRECOND_ABS ? STOP_ABS : STOP_REL;
    SysDesc d;
    memset(&d, 0, sizeof d);
    d.n = n;
    d.ntiles = ntiles;
    d.fmt = FMT_CSRV;
    d.lanes = csrv_default_lanes((double)nnz / n);
    d.stop = stop;
    d.maxit = o->max_iter;
    d.fixed = o->fixed_iters;
    d.prec = PREC_F64;
    d.pair = -1;
    d.tol = o->tol;
    d.rp = A->row_ptr;
    d.col = A->col_idx;
    d.val = A->values;
    d.dinv = dinv;
    d.x = x;
    d.r = vec[0];
    d.u = vec[1];
    d.w = vec[2];
    d.m = vec[3];
    d.nv = vec[4];
    d.z = vec[5];
    d.q = vec[6];
    d.s = vec[7];
    d.p = vec[8];
    d.b = b;
    d.part = part;
    d.st = st;
    PPCG_HIP(hipMemcpyAsync(desc, &d, sizeof d, hipMemcpyHostToDevice, s));
    if (!x0)
        k_na_zero<<<(n + 255) / 256, 256, 0, s>>>(n, x);
    else if (x0 != x)
        PPCG_HIP(hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    PPCG_HIP(hipGetLastError());

    const int remap = PPCG_XCD_REMAP;
    int restarts = 0;
    SysState sh;
    memset(&sh, 0, sizeof sh);
    double rel = 0.0;
    int status = PPCG_OK;
    for (;;) {
        // a start (the first, or a restart from x with x completed first)
        if (restarts > 0)
            launch_x_complete(s, table, count, desc, ntiles);
        // a first start from x0 = 0 needs no pass over A for r0 = b
        launch_pipecg_init(s, table, count, desc, ntiles, restarts == 0 && !x0);
        PPCG_HIP(hipGetLastError());
        double last_norm = -1.0, rate = -1.0;
        int last_iter = 0;
        bool polled = false;
        for (;;) {
            const int want = iters_needed(d, sh, rate, polled, kNaMaxChunk, false);
            int k = 1;
            while (k * 2 <= want)
                k *= 2;
            for (int i = 0; i < k; ++i)
                launch_pipecg_iter(s, table, count, desc, ntiles, remap);
            PPCG_HIP(hipGetLastError());
            PPCG_TRY(na_read_state(s, st, &sh));
            if (sh.done)
                break;
            note_progress(d, sh, &last_norm, &last_iter, &rate);
            polled = true;
        }
        launch_x_complete(s, table, count, desc, ntiles);
        launch_true_resid(s, table, count, desc, ntiles);
        PPCG_HIP(hipGetLastError());
        PPCG_TRY(na_read_state(s, st, &sh));
        const double bn = std::sqrt(sh.bnorm2);
        rel = bn > 0 ? std::sqrt(sh.tnorm2) / bn : std::sqrt(sh.tnorm2);
        const FinalAction act = final_action(*o, sh, restarts, rel, o->tol);
        if (act == FINAL_RESTART) {
            ++restarts;
            sh.done = 0;
            continue;
        }
        status = act == FINAL_STAGNATED ? PPCG_STAGNATED : sh.status;
        break;
    }
    if (info) {
        memset(info, 0, sizeof *info);
        info->struct_size = sizeof *info;
        info->status = (ppcg_status)status;
        info->iters = sh.iter;
        info->restarts = restarts;
        info->rel_resid_true = rel;
        const double bn = std::sqrt(sh.bnorm2);
        info->rel_resid_recur = bn > 0 ? std::sqrt(sh.rr) / bn : std::sqrt(sh.rr);
        info->precond_norm = std::sqrt(sh.uu);
        info->time_ms = now_ms() - t0;
        // fused update: 14 vectors on average (dinv streamed); CSR-vector
        // SpMV: values, columns, row pointers, input and output vectors
        const double bytes = 14.0 * 8.0 * n + 12.0 * (double)nnz + 4.0 * (n + 1) + 16.0 * n;
        info->model_bytes = bytes * sh.iter;
        info->precision = PPCG_FP64;
        info->method = PPCG_METHOD_PIPECG;
    }
    return (ppcg_status)status;
}

}  // namespace
}  // namespace ppcg

using namespace ppcg;

extern "C" ppcg_status ppcg_solve_noalloc(const ppcg_csr *A, const ppcg_options *opt, const double *b,
                                          const double *x0, double *x, ppcg_info *info, void *hip_stream)
{
    clear_error();
    PPCG_TRY(check_options(opt));
    if (!A || A->struct_size != sizeof(ppcg_csr)) {
        set_error("A NULL or struct_size mismatch");
        return PPCG_ERR_INVALID_ARG;
    }
    if (info && info->struct_size != sizeof(ppcg_info)) {
        set_error("info struct_size mismatch");
        return PPCG_ERR_INVALID_ARG;
    }
    if (opt->precision != PPCG_FP64 || opt->method != PPCG_METHOD_PIPECG || opt->vec_mem != PPCG_MEM_DEVICE ||
        opt->spmv_format == PPCG_SPMV_SELL || A->mem != PPCG_MEM_DEVICE) {
        set_error("ppcg_solve_noalloc runs FP64 PIPECG with the CSR-vector SpMV on device arrays only");
        return PPCG_ERR_INVALID_ARG;
    }
    if (A->n < 1 || A->n > kNaMaxRows) {
        set_error("ppcg_solve_noalloc: n = %d outside [1, %d] (the size of its static scratch buffer)", A->n,
                  kNaMaxRows);
        return PPCG_ERR_INVALID_ARG;
    }
    if (A->nnz < A->n || A->nnz >= (int64_t)INT32_MAX) {
        set_error("invalid CSR description (n=%d nnz=%lld)", A->n, (long long)A->nnz);
        return PPCG_ERR_INVALID_ARG;
    }
    const size_t vb = sizeof(double) * (size_t)A->n;
    PPCG_TRY(check_dev_range(A->row_ptr, sizeof(int) * ((size_t)A->n + 1), "row_ptr"));
    PPCG_TRY(check_dev_range(A->col_idx, sizeof(int) * (size_t)A->nnz, "col_idx"));
    PPCG_TRY(check_dev_range(A->values, sizeof(double) * (size_t)A->nnz, "values"));
    PPCG_TRY(check_dev_range(b, vb, "b"));
    PPCG_TRY(check_dev_range(x, vb, "x"));
    if (x0)
        PPCG_TRY(check_dev_range(x0, vb, "x0"));
    // x is iterated in place with 16-byte vector accesses
    if ((uintptr_t)x % 16 != 0 || (uintptr_t)b % 8 != 0 || (x0 && (uintptr_t)x0 % 8 != 0)) {
        set_error("x must be 16-byte aligned, b and x0 8-byte aligned");
        return PPCG_ERR_INVALID_ARG;
    }
    if (x0 && x0 != x && (const double *)x0 < x + A->n && x < (const double *)x0 + A->n) {
        set_error("x0 overlaps x without being equal to it");
        return PPCG_ERR_INVALID_ARG;
    }
    int dev = 0;
    PPCG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) {
        set_error("device %d beyond the %d devices ppcg_solve_noalloc supports", dev, kNaMaxDevices);
        return PPCG_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_na_mu[dev]);
    unsigned char *base = nullptr;
    PPCG_TRY(na_scratch(dev, &base));
    return na_solve(A, opt, b, x0, x, info, (hipStream_t)hip_stream, base);
}
