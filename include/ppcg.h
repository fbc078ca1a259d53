/*
 * ppcg.h -- C ABI of the MI355X (gfx950) Pipelined PCG library.
 *
 * The library solves A x = b for a sparse symmetric positive definite A given
 * in CSR form, with the Jacobi preconditioner, using the pipelined
 * preconditioned conjugate gradient method (PIPECG) of Ghysels and Vanroose
 * as presented by Tiwari & Vadhiyar, "Efficient executions of Pipelined
 * Conjugate Gradient Method on Heterogeneous Architectures", Algorithm 2
 * (Section III-B).  The problem statement follows Sections I, V-A and VI of
 * that paper: A in CSR (Section V-A), a right-hand side b, an initial guess
 * x0, a tolerance and a maximum number of iterations (Section VI), and the
 * Jacobi preconditioner M = diag(A) (Section V-A).
 *
 * Conventions shared by every call:
 *   - Every call returns a ppcg_status.  Nothing aborts, throws or exits
 *     across this ABI; ppcg_last_error() gives a detail message for the most
 *     recent failing call on the calling thread.
 *   - Pointers are plain host or device pointers as stated per argument.
 *     Device pointers are HIP device allocations on the device that was
 *     current when the handle was created (torch tensors' data_ptr() work).
 *   - Work is ordered on the HIP stream given at creation (NULL = the
 *     default stream).  A call returns once its outputs are final.
 *   - Handles are not thread-safe; one handle may be used by one thread at
 *     a time and takes part in at most one solve at a time.  Different
 *     handles (and servers) may be used from different threads at once: the
 *     autotuner's choices and the library's memory releases are shared
 *     safely, and results do not depend on what other threads run.
 *   - Sizes: n >= 1 rows, nnz < 2^31.  Row pointers and column indices are
 *     int32, values float64.
 */
#ifndef PPCG_H
#define PPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppcg_handle ppcg_handle; /* opaque, owned by the library */

typedef enum {
    PPCG_OK = 0,               /* converged (or ran its fixed iterations) */
    PPCG_NOT_CONVERGED = 1,    /* reached max_iter; x holds the last iterate */
    PPCG_BREAKDOWN = 2,        /* gamma <= 0, alpha denominator <= 0 or non-finite scalar */
    PPCG_STAGNATED = 3,        /* recurrence converged, true residual > tol after all restarts */
    PPCG_ERR_INVALID_ARG = -1, /* bad pointer, size, enum or option; outputs untouched */
    PPCG_ERR_BAD_CSR = -2,     /* malformed CSR or missing / non-positive diagonal */
    PPCG_ERR_NOMEM = -3,       /* device or pinned host allocation failed */
    PPCG_ERR_DEVICE = -4,      /* a HIP call failed */
    PPCG_ERR_BUDGET = -5       /* serving: request footprint exceeds the memory budget */
} ppcg_status;

/* Stopping test, evaluated at the top of every iteration (before alpha and
 * beta, Section IV-C). */
typedef enum {
    PPCG_STOP_REL_RESID = 0,  /* sqrt((r,r)) <= tol * ||b||_2 on the recurrence residual;
                                 the final true residual is checked and the solve restarted
                                 from x when it is above tol (default) */
    PPCG_STOP_PRECOND_ABS = 1 /* sqrt((u,u)) < tol, u = M^-1 r: the paper's absolute
                                 preconditioned-residual test (Section VI) */
} ppcg_stop;

typedef enum {
    PPCG_FP64 = 0,        /* every vector, matrix value and scalar in FP64 */
    PPCG_MIXED_FP32 = 1,  /* FP32 matrix values and vectors, FP64 dot products and
                             scalars: one Algorithm 1 sequence on the system scaled by
                             the FP64 residual, with FP64 reliable updates (x64 +=
                             correction, r64 = b - A64 x64, rescaled, direction kept)
                             whenever its residual fell by inner_tol (default 1e-2).
                             Always Algorithm 1, whatever ppcg_options.method says:
                             Algorithm 2's auxiliary recurrences (w, z, s) do not
                             survive FP32 storage.  ppcg_info.method reports it */
    PPCG_MIXED_FP32_VALUES = 2, /* one PIPECG sequence whose SpMVs read FP32 matrix values
                             (FP64 vectors, FP64 accumulation, FP64 dots and scalars),
                             with reliable updates: whenever the residual has dropped by
                             inner_tol (default 1e-3) the FP64 residual b - A x is
                             recomputed with the FP64 values and the pipelined
                             auxiliary vectors are rebuilt from it */
    PPCG_PRECISION_AUTO = 3 /* serving only (ppcg_srv_submit): the server chooses per request by
                             a byte model of one iteration; FP64 PIPECG moves 12 bytes per
                             stored entry + 136 per row.  Systems of at least 262144 rows run
                             PPCG_MIXED_FP32 (Algorithm 1, 8 per entry + 48 per row) when
                             that is at most 70% of FP64's bytes: enough to pay for its two
                             extra launches per iteration.  Systems of at least 65536 rows
                             run PPCG_MIXED_FP32_VALUES (8 per entry + 136 per row) when that
                             is at least 5% below FP64's.  Below 65536 rows launch latency,
                             not bytes, sets the time: PPCG_FP64.  A request run in reduced
                             precision that ends PPCG_STAGNATED, PPCG_BREAKDOWN, or
                             PPCG_NOT_CONVERGED with its refinement budget (max_outer) spent is
                             run again in PPCG_FP64 with the server's method from its last
                             iterate.  ppcg_info reports the precision and method used */
} ppcg_precision;

/* Iteration scheme (ppcg_options.method). */
typedef enum {
    PPCG_METHOD_PIPECG = 0, /* Algorithm 2 (Section III-B): one fused vector update with all
                               dot products, then the SpMV that overlaps their reduction
                               (default) */
    PPCG_METHOD_PCG = 1     /* Algorithm 1 (Section III-A): classic PCG; two launches per
                               iteration, each ending in a reduction the next launch waits
                               for.  With PPCG_FP64, PPCG_MIXED_FP32_VALUES (FP32 values,
                               reliable updates r = b - A x keeping the direction).
                               PPCG_MIXED_FP32 always runs Algorithm 1 */
} ppcg_method;

typedef enum { PPCG_MEM_DEVICE = 0, PPCG_MEM_HOST = 1 } ppcg_mem;

/* SpMV formats the autotuner chooses from (ppcg_options.spmv_format). */
typedef enum {
    PPCG_SPMV_AUTO = 0,      /* autotune: time the candidates on this matrix */
    PPCG_SPMV_SELL = 1,      /* SELL-C-sigma, one lane per row, C = 64 */
    PPCG_SPMV_CSR_VECTOR = 2 /* CSR, a group of lanes (2..64) per row */
} ppcg_spmv_format;

/* A in CSR.  Caller-owned; read only during ppcg_create (the library keeps
 * its own device copy, so the arrays may be freed once ppcg_create returns).
 * Requirements: row_ptr[0] = 0, row_ptr non-decreasing, row_ptr[n] = nnz,
 * 0 <= col_idx < n, columns strictly ascending within a row, every row
 * stores a finite diagonal entry > 0, all values finite.  Symmetry and
 * positive definiteness are not checked (a matrix that is not SPD ends in
 * PPCG_BREAKDOWN or PPCG_NOT_CONVERGED). */
typedef struct {
    size_t struct_size;      /* sizeof(ppcg_csr) */
    int32_t n;               /* rows = columns */
    int64_t nnz;             /* stored entries */
    const int32_t *row_ptr;  /* [n + 1] */
    const int32_t *col_idx;  /* [nnz] */
    const double *values;    /* [nnz] */
    ppcg_mem mem;            /* where the three arrays live */
} ppcg_csr;

/* ppcg_options.flags bits (any other bit is ERR_INVALID_ARG). */
#define PPCG_FLAG_BORROW_INPUTS 1u /* serving (ppcg_srv_create's options): requests reference the
                                      caller's A and b arrays instead of copying them; they must
                                      stay valid and unchanged until ppcg_srv_poll reports the
                                      request ready.  Ignored elsewhere */
#define PPCG_FLAG_SELL_COL16 2u    /* SELL: read 16-bit column offsets from the row whenever all
                                      fit, without timing them against 32-bit columns (by default
                                      both are timed at create time and the faster is kept).
                                      Read by ppcg_create only, like the format itself */
#define PPCG_FLAG_SELL_COL32 4u    /* SELL: always read 32-bit columns (not with SELL_COL16) */
#define PPCG_FLAG_SELL_VALUE_TABLE 8u /* SELL: when the matrix has at most 256 distinct values (the
                                         padding's 0.0 included), the PIPECG SpMV with FP64
                                         values reads a one-byte index per stored entry into a
                                         table of them, without timing it against the 8-byte
                                         values (by default both are timed at create time and the
                                         faster is kept).  Exact: the same values multiply.  Read
                                         by ppcg_create only */
#define PPCG_FLAG_SELL_FULL_VALUES 16u /* SELL: never build the value table (not with
                                          SELL_VALUE_TABLE) */
#define PPCG_FLAG_ITER_FUSED 32u   /* FP64 PIPECG on SELL storage: one launch per iteration (the
                                      SpMV, the reduction of the previous dot products with the
                                      scalar recurrences, and the fused vector updates with n kept
                                      in registers), without timing it against the two-launch form
                                      (by default, for systems above 4096 rows, both are timed at
                                      create time and the faster is kept).  The dot products are
                                      associated over 2048-row tiles instead of 512-row ones, so
                                      results differ from the two-launch form by rounding.  Read by
                                      ppcg_create only */
#define PPCG_FLAG_ITER_TWO_LAUNCH 64u /* always two launches per iteration (not with ITER_FUSED) */
#define PPCG_FLAG_SELL_SHARED_OFFSETS 128u /* SELL with rows in their own order: when the column
                                      offsets (column minus row) of the 64 rows of every chunk,
                                      merged, form one list (stencils in natural order; the chunk
                                      then stores that many slots), the PIPECG SpMV with FP64
                                      vectors (FP64 or FP32 values) reads the chunk's one offset
                                      list instead of a column per entry, without timing it
                                      against the per-entry columns (by default, unless SELL_COL16
                                      or SELL_COL32 pins a column layout, both are timed at create
                                      time and the faster is kept).  Rows missing an offset
                                      of the list hold an explicit zero there, so the products and
                                      their order are those of the CSR rows.  Read by ppcg_create
                                      only */
#define PPCG_FLAG_SELL_NO_SHARED_OFFSETS 256u /* SELL: never read shared offset lists (not with
                                                 SELL_SHARED_OFFSETS) */

/* Solver options; initialise with ppcg_default_options(). */
typedef struct {
    size_t struct_size;      /* sizeof(ppcg_options) */
    double tol;              /* stopping tolerance (default 1e-8) */
    int32_t max_iter;        /* maximum total iterations (default 10000, the paper's) */
    int32_t fixed_iters;     /* > 0: run exactly this many iterations, ignore tol and
                                max_iter; stop early only on breakdown or gamma == 0 */
    int32_t max_restarts;    /* restarts from x allowed (default 3) */
    ppcg_stop stop;          /* default PPCG_STOP_REL_RESID */
    ppcg_precision precision;/* default PPCG_FP64 */
    ppcg_mem vec_mem;        /* where b, x0 and x live (default PPCG_MEM_DEVICE) */
    ppcg_spmv_format spmv_format; /* default PPCG_SPMV_AUTO */
    int32_t graph_iters;     /* iterations per captured HIP graph; 0 = automatic */
    double inner_tol;        /* residual reduction between reliable updates:
                                PPCG_MIXED_FP32 (0 = 1e-2), PPCG_MIXED_FP32_VALUES
                                (0 = 1e-3) */
    int32_t max_outer;       /* mixed precision: maximum refinement steps / reliable
                                updates (default 30) */
    ppcg_method method;      /* default PPCG_METHOD_PIPECG */
    uint32_t flags;          /* PPCG_FLAG_* bits, default 0 */
} ppcg_options;

/* Per-solve report. */
typedef struct {
    size_t struct_size;      /* sizeof(ppcg_info) */
    ppcg_status status;
    int32_t iters;           /* PIPECG iterations (x-updates); total inner iterations in
                                mixed precision */
    int32_t outer_iters;     /* refinement steps (PPCG_MIXED_FP32) or reliable updates
                                (PPCG_MIXED_FP32_VALUES), else 0 */
    int32_t restarts;        /* restarts from x (true residual above tol, or breakdown) */
    double rel_resid_true;   /* ||b - A x||_2 / ||b||_2 in FP64 at exit */
    double rel_resid_recur;  /* sqrt((r,r)) / ||b|| of the recurrence at exit */
    double precond_norm;     /* sqrt((u,u)) at exit */
    double time_ms;          /* wall time of the solve on its stream */
    double model_bytes;      /* algorithmic HBM bytes moved by the iterations */
    ppcg_precision precision;/* precision the solve ran in (the server's choice for
                                PPCG_PRECISION_AUTO; PPCG_FP64 after an automatic rerun) */
    ppcg_method method;      /* iteration scheme the solve ran with */
} ppcg_info;

/* Static description of a handle's matrix as the library stores it. */
typedef struct {
    size_t struct_size;      /* sizeof(ppcg_matrix_info) */
    int32_t n;
    int64_t nnz;
    int64_t nnz_stored;      /* entries stored including SELL padding */
    ppcg_spmv_format format; /* format chosen (never AUTO) */
    int32_t sell_c;          /* SELL chunk height */
    int32_t sell_sigma;      /* SELL sorting window (1 = unsorted) */
    int32_t lanes_per_row;   /* CSR-vector group size */
    int32_t tile_rows;       /* rows per workgroup tile */
    double bytes_per_iter;   /* algorithmic HBM bytes of one iteration (both kernels) of
                                the handle's current method (opt.method) */
    double bytes_vma;        /* algorithmic bytes of one vector-update launch (PIPECG: fused
                                VMA+PC+dots, 14 vectors on average, x being read and
                                written every other launch; PCG: 8 vectors; one fewer
                                when diag_const) */
    double bytes_spmv;       /* algorithmic bytes of one SpMV launch (matrix plus 2 vectors;
                                PCG: plus 4, the direction update being fused into it) */
    double device_bytes;     /* device memory held by the handle */
    double setup_ms;         /* time spent in ppcg_create (validation, conversion, tuning) */
    int32_t col_index_bytes; /* bytes per stored column index the iteration's SpMV reads: 2 when
                                every SELL column fits a 16-bit offset from its row, 0 when the
                                PIPECG SpMV with FP64 vectors reads the chunks' shared offset
                                lists (PPCG_FLAG_SELL_SHARED_OFFSETS), else 4 */
    int32_t diag_const;      /* 1: every diagonal entry is equal; the fused update then reads
                                the inverse diagonal as one cached value, not a vector */
    int32_t value_bytes;     /* bytes per stored value the iteration's SpMV reads: 1 with the
                                value table (FP64 PIPECG), 4 with FP32 values, else 8 */
    int32_t distinct_values; /* entries of the value table (0 when there is none) */
    int32_t iter_launches;   /* launches per iteration of the handle's current method and
                                precision: 1 for FP64 PIPECG in the single-launch form
                                (bytes_per_iter then omits n's write and read, 16 bytes per
                                row), else 2 */
} ppcg_matrix_info;

/* Fill *opt with the defaults listed above. */
ppcg_status ppcg_default_options(ppcg_options *opt);

/* Create a solver handle for matrix A (Section V-A: CSR input, Jacobi
 * preconditioner).  Validates A on the device, builds dinv = 1 / diag(A),
 * converts A to the SpMV format (autotuned when spmv_format is AUTO), keeps
 * an FP32 copy of the values when opt->precision is PPCG_MIXED_FP32, and
 * allocates the solver vectors.  hip_stream: a hipStream_t (NULL = default
 * stream).  On success *out receives the handle; on error *out is set to NULL
 * and nothing is leaked.  Errors: PPCG_ERR_INVALID_ARG (null pointers,
 * struct_size mismatch, n < 1, nnz out of range, bad options),
 * PPCG_ERR_BAD_CSR (see ppcg_csr), PPCG_ERR_NOMEM, PPCG_ERR_DEVICE. */
ppcg_status ppcg_create(const ppcg_csr *A, const ppcg_options *opt, void *hip_stream,
                        ppcg_handle **out);

/* Replace the handle's options (tolerance, limits, stop mode, precision...).
 * Switching to PPCG_MIXED_FP32 builds the FP32 copy on first use. */
ppcg_status ppcg_set_options(ppcg_handle *h, const ppcg_options *opt);

/* Solve A x = b with Algorithm 2 (PIPECG).  b: [n] FP64, x0: [n] FP64 or NULL
 * (NULL = zero initial guess; x0 may alias x), x: [n] FP64 output; all three
 * in opt.vec_mem memory and owned by the caller.  info may be NULL.
 * Returns the solve status (also in info->status).  PPCG_NOT_CONVERGED,
 * PPCG_BREAKDOWN and PPCG_STAGNATED still write the last iterate to x and
 * fill info.  Argument errors leave x untouched. */
ppcg_status ppcg_solve(ppcg_handle *h, const double *b, const double *x0, double *x, ppcg_info *info);

/* Solve count independent systems in one batched launch sequence: every
 * PIPECG iteration of all unconverged systems runs over a table of (system,
 * row tile) work items, captured in HIP graphs (one launch per iteration for
 * the systems in the single-launch form, a fused-update launch and an SpMV
 * launch for the others); converged systems leave the table between graph
 * launches.  hs: [count] distinct handles on one device; their streams may
 * differ: the batch waits for the work queued on every handle's stream
 * before it reads b[i] and x0[i], and returns once x[i] is written.  b, x0,
 * x: [count] arrays of per-system pointers as in ppcg_solve (x0[i] or x0
 * itself may be NULL).  infos: [count] or NULL.  Returns PPCG_OK when the
 * batch ran; per-system outcomes are in infos[i].status.  Each system's
 * result is bitwise identical to solving it alone with ppcg_solve.
 * Resources: hs[0] keeps the batch's engine (device buffers for count
 * systems, its streams and captured graphs) until it leads a batch of more
 * systems or is destroyed, so that the next batch it leads starts without
 * allocating or capturing; an error during a batch releases them. */
ppcg_status ppcg_solve_batch(int32_t count, ppcg_handle *const *hs, const double *const *b,
                             const double *const *x0, double *const *x, ppcg_info *infos);

/* ppcg_solve without a handle and without allocating, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Solves A x = b with Algorithm 2, FP64,
 * Jacobi, on the caller's CSR arrays in device memory (A->mem must be
 * PPCG_MEM_DEVICE; the CSR requirements of ppcg_csr apply and are checked on
 * the device), with the CSR-vector SpMV; b, x0 (NULL = 0; may equal x) and x
 * are device [n] FP64 arrays, x 16-byte aligned; opt: PPCG_FP64,
 * PPCG_METHOD_PIPECG, vec_mem PPCG_MEM_DEVICE, spmv_format AUTO or
 * CSR_VECTOR; tol, max_iter, fixed_iters, max_restarts and stop as for
 * ppcg_solve.  Work is ordered on hip_stream (NULL = default stream); the call
 * returns once x and info are final.
 * Memory: every buffer the kernels need besides the caller's (nine solver
 * vectors, the inverse diagonal, partial sums, work table, state) lives in
 * one static device array of about 40 MiB that each device holds from the
 * library's first use of it until the process ends; the call makes no
 * allocation (no hipMalloc, hipHostMalloc or graph).  Limit: n <= 524288
 * rows; larger n is PPCG_ERR_INVALID_ARG.  The array is shared by all calls
 * on one device and keeps the last call's contents: calls on one device are
 * serialized by a lock inside the library; concurrent calls on one device
 * from different processes would race.
 * Result: bitwise equal to ppcg_solve on a handle created from the same
 * arrays with spmv_format = PPCG_SPMV_CSR_VECTOR and the same options.
 * Errors as for ppcg_create and ppcg_solve; argument errors leave x untouched. */
ppcg_status ppcg_solve_noalloc(const ppcg_csr *A, const ppcg_options *opt, const double *b, const double *x0,
                               double *x, ppcg_info *info, void *hip_stream);

/* y = A x with the handle's SpMV kernel (Algorithm 2's SpMV step, A in the
 * stored format chosen at creation).  x, y: [n] FP64 in opt.vec_mem memory,
 * caller-owned, must not alias.  Each row is summed in the CSR column order
 * (SELL format) or by a fixed lane-strided tree (CSR-vector format). */
ppcg_status ppcg_spmv(ppcg_handle *h, const double *x, double *y);

/* Describe the stored matrix and the algorithmic byte model. */
ppcg_status ppcg_get_matrix_info(const ppcg_handle *h, ppcg_matrix_info *mi);

/* Device bytes a handle for an n x n matrix with nnz entries would hold
 * (matrix in its SpMV format with padding estimate, dinv, the eleven solver
 * vectors, b, partials and state; plus the FP32 copy when mixed).  Used for
 * admission by footprint.  Returns 0 for invalid sizes. */
double ppcg_footprint_bytes(int32_t n, int64_t nnz, ppcg_precision precision);

/* Measure the two kernels of the iteration (Algorithm 2's fused vector
 * updates + preconditioner + dot products, and its SpMV) over `iters`
 * iterations on the handle's stream, each launch bracketed by HIP events.
 * A handle in the single-launch form (ppcg_matrix_info.iter_launches = 1 with
 * PPCG_FP64 PIPECG) times its one kernel: *ms_vma receives its average
 * duration and *ms_spmv 0.
 * Runs the initialisation first, so the vectors hold a real iterate.
 * With opt.method = PPCG_METHOD_PCG the two streaming kernels of Algorithm 1
 * are timed instead (vector updates + preconditioner + dot-product partials;
 * SpMV with the direction update and the (s, p) partials); the per-system
 * reductions between them run but are not included.
 * ms_vma, ms_spmv: average launch duration in milliseconds (host pointers). */
ppcg_status ppcg_time_kernels(ppcg_handle *h, const double *b, int32_t iters, double *ms_vma,
                              double *ms_spmv);

/* Release the handle and all its device memory.  NULL-safe.  Must not be
 * called while a solve using the handle is in flight. */
ppcg_status ppcg_destroy(ppcg_handle *h);

/* Static string naming a status. */
const char *ppcg_status_str(ppcg_status s);

/* Detail message of the last failing call on this thread ("" if none). */
const char *ppcg_last_error(void);

/* ---------------------------------------------------------------------------
 * Row split and 2-D decomposition (Section IV-C, "Performance Modelling" and
 * "Data Decomposition").  The paper divides A between processing units in
 * proportion to the speed each shows on the same SpMV, then splits every
 * unit's entries into those that need only the unit's own piece of the
 * vector (its SpMV part 1) and those that need elements owned by others
 * (part 2, after they have been copied in).  Here the units are devices of
 * a multi-GPU (or host + GPU) run; these calls plan the split and hold one
 * unit's share with its two-part SpMV.  The exchange between units is not
 * part of the library.
 * ------------------------------------------------------------------------- */

/* Rows per unit.  times[k] (> 0, seconds): unit k's time for the same SpMV
 * over all nnz entries; its speed s_k = nnz / t_k and share r_k = s_k / sum s.
 * Unit k gets the rows [row_begin[k], row_begin[k+1]); each boundary before
 * the last is the most leading row count whose non-zeros number at most
 * nnz * (r_1 + ... + r_k) (equal or slightly fewer, as in the paper, which
 * has two units); the last unit takes the rest.  row_ptr: host [n + 1];
 * times: host [parts]; row_begin: host [parts + 1], written.  Host only. */
ppcg_status ppcg_split_rows(int32_t n, const int32_t *row_ptr, int32_t parts, const double *times,
                            int32_t *row_begin);

typedef struct ppcg_shard ppcg_shard; /* opaque, owned by the library */

typedef struct {
    size_t struct_size;      /* sizeof(ppcg_shard_info) */
    int32_t row_begin;       /* the unit's rows are [row_begin, row_end) */
    int32_t row_end;
    int64_t nnz_local;       /* nnz1: entries whose column is also in [row_begin, row_end) */
    int64_t nnz_remote;      /* nnz2: the other entries */
    int32_t halo;            /* distinct remote columns = length of the halo vector */
    int32_t boundary_rows;   /* rows with at least one remote entry */
    double bytes_part1;      /* algorithmic bytes of part 1 (matrix, input, output) */
    double bytes_part2;      /* algorithmic bytes of part 2 (matrix, halo, output update) */
    double halo_bytes;       /* bytes the unit receives per SpMV (8 per halo entry) */
} ppcg_shard_info;

/* One unit's share of A: rows [row_begin, row_end) of the n x n CSR matrix A
 * (host or device arrays, read during the call only; A's CSR requirements
 * apply to these rows, no diagonal is needed).  Part 1 is stored with local
 * columns (0 .. rows-1); part 2 with columns renumbered to the halo vector,
 * which lists the distinct remote columns in ascending order.  Work is
 * ordered on hip_stream.  Errors: ERR_INVALID_ARG (range, pointers),
 * ERR_BAD_CSR, ERR_NOMEM. */
ppcg_status ppcg_shard_create(const ppcg_csr *A, int32_t row_begin, int32_t row_end, void *hip_stream,
                              ppcg_shard **out);
ppcg_status ppcg_shard_get_info(const ppcg_shard *s, ppcg_shard_info *info);
/* cols: host [halo], receives the global column of every halo entry. */
ppcg_status ppcg_shard_halo_columns(const ppcg_shard *s, int32_t *cols);
/* x_halo[k] = x_global[cols[k]] on the device: the halo a unit would receive
 * from the others, taken here from a global vector.  Device pointers. */
ppcg_status ppcg_shard_gather(ppcg_shard *s, const double *x_global, double *x_halo);
/* y = A_rows x in two parts: parts & 1 writes y = (part 1) x_local, parts & 2
 * adds (part 2) x_halo to y.  Row i's part-1 and part-2 entries are each
 * summed in stored column order and the two sums added.  x_local: device
 * [rows], x_halo: device [halo], y: device [rows], not aliasing x_local. */
ppcg_status ppcg_shard_spmv(ppcg_shard *s, const double *x_local, const double *x_halo, double *y,
                            int32_t parts);
/* Average durations (ms, HIP events attached to each launch) over iters
 * rounds of part 1, the halo gather from x_global, and part 2. */
ppcg_status ppcg_shard_time(ppcg_shard *s, const double *x_global, const double *x_local, double *x_halo,
                            double *y, int32_t iters, double *ms_part1, double *ms_gather, double *ms_part2);
ppcg_status ppcg_shard_destroy(ppcg_shard *s); /* NULL-safe */

/* ---------------------------------------------------------------------------
 * Host cores + GPU together (Section IV): Algorithm 2 in one of the paper's
 * three execution schemes.  Alpha and beta are always computed on the host.
 *
 * PPCG_HYBRID_3 (Section IV-C, data parallel).  Setup times five SpMVs over
 * all of A on the host threads and on the GPU, splits the rows with the
 * performance model (ppcg_split_rows: rows [0, n_cpu) on the host, the rest
 * on the GPU) and builds both sides' 2-D decomposition.  Each iteration: the
 * m entries each side needs from the other move (device <-> pinned host
 * memory) while both sides update q, s, p, x, r, u and compute SpMV part 1;
 * part 2 runs once the copy has arrived; then z, w, m and the dot products;
 * the host adds both sides' partial sums.
 *
 * PPCG_HYBRID_1 and PPCG_HYBRID_2 (Sections IV-A, IV-B, task parallel): every
 * row lives on the GPU, which runs all vector updates, the preconditioner and
 * the SpMV.  Hybrid-1 copies w, r and u to pinned host memory after the
 * updates, overlapping the GPU's preconditioner and SpMV, and host threads
 * form gamma, delta and the norms from them.  Hybrid-2 copies only n: the host
 * keeps full-length copies of z, q, s, r, u, w, m and repeats their updates,
 * q, s, r, u and gamma while n is in flight, then z, w, m and delta.
 * ------------------------------------------------------------------------- */
typedef struct ppcg_hybrid ppcg_hybrid; /* opaque, owned by the library */

typedef enum {
    PPCG_HYBRID_1 = 1, /* task parallel: w, r, u copied each iteration, dot products on the host */
    PPCG_HYBRID_2 = 2, /* task parallel: n copied each iteration, host repeats the updates */
    PPCG_HYBRID_3 = 3  /* data parallel: performance-model row split, 2-D decomposition */
} ppcg_hybrid_scheme;

typedef struct {
    size_t struct_size;       /* sizeof(ppcg_hybrid_info) */
    int32_t n_cpu;            /* rows [0, n_cpu) iterate on the host */
    int32_t n_gpu;            /* rows [n_cpu, n) iterate on the GPU */
    int32_t host_threads;
    double t_cpu_spmv_ms;     /* performance model: one SpMV over all of A on the host threads */
    double t_gpu_spmv_ms;     /* ... and on the GPU */
    int64_t nnz_cpu_local;    /* host part 1 / part 2 entries */
    int64_t nnz_cpu_remote;
    int64_t nnz_gpu_local;    /* GPU part 1 / part 2 entries */
    int64_t nnz_gpu_remote;
    int32_t halo_to_cpu;      /* m entries copied GPU -> host per iteration (Hybrid-3) */
    int32_t halo_to_gpu;      /* m entries copied host -> GPU per iteration (Hybrid-3) */
    ppcg_hybrid_scheme scheme;
    double copy_bytes_per_iter; /* device <-> host bytes per iteration (both directions) */
} ppcg_hybrid_info;

/* A: host CSR (read during the call).  opt: PPCG_FP64, PPCG_METHOD_PIPECG,
 * vec_mem = PPCG_MEM_HOST (b, x0, x are host arrays); tol, max_iter,
 * fixed_iters, max_restarts and stop as for ppcg_solve.  scheme: one of
 * ppcg_hybrid_scheme.  host_threads: 1..256.  Hybrid-3: cpu_share < 0 splits
 * by the performance model; 0 <= cpu_share <= 1 gives the host that share of
 * the non-zeros instead (same row rule).  Hybrid-1/2: cpu_share must be < 0
 * (every row is on the GPU).  Errors: ERR_INVALID_ARG, ERR_BAD_CSR,
 * ERR_NOMEM, ERR_DEVICE. */
ppcg_status ppcg_hybrid_create(const ppcg_csr *A, const ppcg_options *opt, ppcg_hybrid_scheme scheme,
                               int32_t host_threads, double cpu_share, void *hip_stream, ppcg_hybrid **out);
ppcg_status ppcg_hybrid_get_info(const ppcg_hybrid *hy, ppcg_hybrid_info *info);
/* b: host [n]; x0: host [n] or NULL (= 0); x: host [n], written; info may be
 * NULL.  Returns the solve status as ppcg_solve does. */
ppcg_status ppcg_hybrid_solve(ppcg_hybrid *hy, const double *b, const double *x0, double *x, ppcg_info *info);
ppcg_status ppcg_hybrid_destroy(ppcg_hybrid *hy); /* NULL-safe */

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching solve server.  Two threads owned by the
 * server prepare queued requests, taken first-come first-served (matrix
 * copied to the device, validated and laid out, right-hand side staged),
 * and hand them over as they become ready, while the sum
 * of the device footprints (ppcg_footprint_bytes) of the requests it holds
 * stays within the budget, and releases the memory of retired ones; both
 * overlap with the iterations of the active requests.  Prepared requests
 * join the batched iteration at the next graph boundary and leave it when
 * they finish, so requests that arrive while others run overlap with them on
 * the device.  Each request's arithmetic is independent of the others in the
 * mix: its result is bitwise identical to a solo ppcg_solve of the same
 * request with the same options.  The calls on one server must not overlap
 * (one calling thread at a time).
 * ------------------------------------------------------------------------- */
typedef struct ppcg_server ppcg_server;

/* Create a server on the current device with a device-memory budget in
 * bytes (0 = 80% of the free device memory).  opt supplies defaults for
 * requests.  The server takes no stream: its inputs and results are host
 * arrays, and it orders its device work on streams of its own. */
ppcg_status ppcg_srv_create(const ppcg_options *opt, double budget_bytes, ppcg_server **out);

/* Queue a request.  A: host CSR; b: host [n] FP64; both copied before
 * returning, or referenced until the request is polled ready when the server
 * was created with PPCG_FLAG_BORROW_INPUTS.  tol: this request's tolerance;
 * precision: any ppcg_precision,
 * PPCG_PRECISION_AUTO included.  *req_id receives the request's id.
 * PPCG_ERR_BUDGET when the request could never fit the budget. */
ppcg_status ppcg_srv_submit(ppcg_server *s, const ppcg_csr *A, const double *b, double tol,
                            ppcg_precision precision, int64_t *req_id);

/* Advance the server: admit the prepared requests, run one graph chunk of
 * iterations over every active request, retire finished ones.  With no
 * active request it first waits until a queued request is prepared (or has
 * failed on its own).  *active and *queued (may be NULL) receive the counts
 * after the step; queued counts the requests not yet admitted.  A device
 * error met while preparing a request is returned by the next step. */
ppcg_status ppcg_srv_step(ppcg_server *s, int32_t *active, int32_t *queued);

/* Fetch a finished request.  Returns PPCG_NOT_CONVERGED with *ready = 0 when
 * it is still queued or running.  When *ready = 1, x (host [n], may be NULL)
 * receives the solution, info (may be NULL) the report, and the request's
 * memory is released. */
ppcg_status ppcg_srv_poll(ppcg_server *s, int64_t req_id, int32_t *ready, double *x, ppcg_info *info);

/* Destroy the server, dropping unfinished requests.  NULL-safe. */
ppcg_status ppcg_srv_destroy(ppcg_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PPCG_H */
