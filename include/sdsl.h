/*
 * sdsl.h - C ABI of the MI355X (gfx950) preconditioned Krylov solver for
 * interior-point-method linear systems.
 *
 * The method is that of "SDSL-Solver: Scalable Distributed Sparse Linear
 * Solvers for Large-Scale Interior Point Methods" (arXiv 2604.23979): at every
 * IPM iteration a sparse system M x = b (Sec. 2.1, Eq. (schur); the system of
 * each interior-point iteration is the input of Alg. 1) is solved by a
 * preconditioned Krylov method (Sec. 2.2, right preconditioning: PCG,
 * GMRES(m), BiCGSTAB, GCR(m)) with either
 *   - a block-Jacobi preconditioner (Sec. 2.3): contiguous row blocks, each
 *     diagonal block filtered (Sec. 3.2, Eq. (filter)), diagonally corrected
 *     (Sec. 3.3, Eq. (diagcorr)) and ILU(0) or completely LU factored
 *     (Sec. 3.1), optionally after MC64 matching and scaling (Alg. 3); or
 *   - a bordered-block-diagonal (BBD) preconditioner (Sec. 2.4): factored
 *     interior blocks coupled through a dense Schur complement of the border.
 * Preconditioners stay resident between calls so that consecutive IPM systems
 * reuse them (Sec. 3.4).  Several handles on one stream can share kernel
 * launches (sdsl_group_*).
 *
 * All arrays named "device" live in GPU memory of the current HIP device;
 * "host" arrays live in CPU memory.  Every call returns an sdsl_status and
 * never aborts or throws; sdsl_last_error() gives a readable reason.  A handle
 * stays usable after any error except SDSL_E_DEVICE.  Handles are not
 * thread-safe; distinct handles may be used from distinct threads.
 * Int32 indices are used internally: n and nnz must be below 2^31.
 */
#ifndef SDSL_H
#define SDSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDSL_ABI_VERSION 2

typedef struct sdsl_ctx* sdsl_handle;

typedef enum {
    SDSL_OK = 0,
    SDSL_E_INVALID = 1,       /* bad argument: NaN/Inf, unsorted or duplicate
                                 columns, missing diagonal, bad partition     */
    SDSL_E_STRUCTURE = 2,     /* BBD: matrix not in bordered block form        */
    SDSL_E_NOMEM = 3,         /* device allocation failed                      */
    SDSL_E_BREAKDOWN = 4,     /* factorisation pivot or Krylov breakdown       */
    SDSL_E_NOT_CONVERGED = 5, /* tolerance not reached within the limits      */
    SDSL_E_DEVICE = 6,        /* HIP runtime error; the handle is unusable     */
    SDSL_E_STATE = 7          /* call not valid in the handle's state          */
} sdsl_status;

typedef enum { SDSL_BJ = 0, SDSL_BBD = 1 } sdsl_method;           /* Sec. 2.3 / 2.4 */

/* Sparse filter of Sec. 3.2.  MIN is Eq. (filter): drop a_ij (i != j) iff
 * |a_ij| < tau |a_ii| and |a_ij| < tau |a_jj|.  GEOMEAN drops iff
 * a_ij^2 < tau^2 |a_ii a_jj|, which is Eq. (filter) after symmetric scaling
 * to a unit diagonal.  Diagonals are always kept; the diagonals used in the
 * test are those of the unfiltered matrix. */
typedef enum { SDSL_FILTER_NONE = 0, SDSL_FILTER_MIN = 1, SDSL_FILTER_GEOMEAN = 2 } sdsl_filter;

/* Diagonal correction of Sec. 3.3 (bit flags, applied to the preconditioner
 * only).  DELTA is Eq. (diagcorr): p_ii += delta * sign(p_ii), sign(0) = +1.
 * DROPSUM adds sign(p_ii) * (sum of |a_ij| dropped by the filter in row i).
 * Both together add sign(p_ii) * (delta + dropsum_i). */
enum { SDSL_DIAG_DELTA = 1u, SDSL_DIAG_DROPSUM = 2u };

/* What to do when ILU(0) meets a bad pivot (non-positive in SPD mode,
 * |u_ii| < 1e-14 |p_ii| otherwise); the paper states no pivot rule, so these
 * are this library's breakdown policies.  FAIL returns SDSL_E_BREAKDOWN;
 * REPLACE replaces the pivot by its corrected diagonal; SHIFT refactors the
 * block with every diagonal raised to d + a*d for a = shift0, 2*shift0, ...
 * up to 48 doublings: a shifted incomplete factorisation (Manteuffel, Math.
 * Comp. 34 (1980)), not the small absolute correction of Eq. (diagcorr). */
typedef enum { SDSL_PIVOT_FAIL = 0, SDSL_PIVOT_REPLACE = 1, SDSL_PIVOT_SHIFT = 2 } sdsl_pivot;

/* Krylov methods (Sec. 2.2; Sec. 4.3 pairs BiCGSTAB with block Jacobi and
 * GCR with BBD): PCG for SPD systems; GMRES(restart), BiCGSTAB and
 * GCR(restart) with right preconditioning.  BiCGSTAB runs with the
 * block-Jacobi preconditioner in FP64; one of its iterations makes two
 * products and two applies.  GCR (Eisenstat, Elman and Schultz 1983) runs
 * in FP64 with either preconditioner; it keeps restart directions and
 * their products, orthonormal products within a cycle, and stops with
 * SDSL_E_BREAKDOWN when a new direction adds nothing to the cycle's space. */
typedef enum { SDSL_PCG = 0, SDSL_GMRES = 1, SDSL_BICGSTAB = 2, SDSL_GCR = 3 } sdsl_krylov;

/* FP64: every step in FP64.
 * FP32_IR: the SpMV and the preconditioner apply run in FP32 (FP32 operator
 * values and factors, products accumulated in FP32) inside an FP64
 * refinement loop: the recurrence vectors, the solution update, the low-rank
 * term and its border correction stay FP64, and at each refinement point
 * (the recurrence residual fell by refine_delta, met the tolerance, or
 * refine_every iterations passed) the true residual is formed in FP64 and
 * replaces the recurrence one, which continues with its search direction
 * (reliable updating).  When the refinement points stop halving the true
 * residual the rest is solved in FP64 (sdsl_info.rf_*).
 * FP32_IR_RESTART: classical refinement; every step restarts the inner PCG
 * on the current residual and stops it at inner_tol (or after refine_every
 * iterations); an inner solve that breaks down is discarded and the rest is
 * solved in FP64. */
typedef enum { SDSL_FP64 = 0, SDSL_FP32_IR = 1, SDSL_FP32_IR_RESTART = 2 } sdsl_precision;

/* Factorisation of each filtered, corrected block (Sec. 3.1: ILU(0) for
 * block Jacobi, complete LU for BBD; Sec. 3.2 Alg. 2: a complete
 * factorisation of the filtered matrix).  COMPLETE: LU without pivoting of
 * the whole block, i.e. elimination over the block's symbolic fill pattern
 * (found on the host, rows merged in natural order; no fill-reducing
 * ordering), numerically by the same in-block elimination as ILU(0); in
 * SPD mode its U is D L^T, the LU form of the complete Cholesky factor.
 * The breakdown policy applies as for ILU(0).  nnz_kept then counts the
 * factor's entries (fill included); the fill is symbolic analysis of the
 * filtered pattern, repeated by refactor, and it is not part of
 * sdsl_footprint_bytes. */
typedef enum { SDSL_FACT_ILU0 = 0, SDSL_FACT_COMPLETE = 1 } sdsl_factor;

typedef enum { SDSL_MEM_DEVICE = 0, SDSL_MEM_HOST = 1 } sdsl_mem;

/* Square sparse matrix in CSR: row_ptr[n+1] (int64), col[nnz] (int32,
 * strictly increasing within a row, diagonal present), val[nnz] (double).
 * `mem` says where the three arrays live. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
    sdsl_mem mem;
} sdsl_csr;

/* Contiguous row blocks (Sec. 2.3, the row partition): block_ptr is a HOST array of
 * nblocks+1 increasing row indices with block_ptr[0] = 0 and
 * block_ptr[nblocks] = n - n_border.  For BBD the n_border trailing rows are
 * the border (Sec. 2.4); for BJ n_border must be 0. */
typedef struct {
    int32_t nblocks;
    const int32_t* block_ptr;
    int32_t n_border;
} sdsl_partition;

/* Optional low-rank operator term: the operator becomes M + U diag(c) U^T
 * with U an n x k CSR matrix (dense columns of the constraint matrix kept
 * apart, Sec. 2.1).  The preconditioner is built from M alone.  Arrays live
 * where U.mem says; c has k entries in the same memory. */
typedef struct {
    int32_t k;
    sdsl_csr U;          /* n x k: U.n = n rows, columns 0..k-1             */
    const double* c;
} sdsl_lowrank;

typedef struct {
    sdsl_method method;
    sdsl_filter filter;
    double tau;            /* filter threshold (Sec. 3.2; 1e-3 typical)      */
    uint32_t diag_flags;   /* SDSL_DIAG_* bits                               */
    double delta;          /* Eq. (diagcorr) delta (paper: 1e-12 typical)    */
    sdsl_pivot pivot;      /* ILU(0) breakdown policy                        */
    double shift0;         /* first relative shift of SDSL_PIVOT_SHIFT       */
    int32_t spd;           /* 1: symmetric positive definite mode            */
    sdsl_krylov krylov;
    int32_t restart;       /* GMRES(m) / GCR(m) restart length, in [1, 63]   */
    int32_t max_iter;      /* Krylov iterations (all inner iterations)       */
    sdsl_precision precision;
    double inner_tol;      /* FP32_IR: relative tolerance of each inner solve */
    int32_t max_outer;     /* FP32_IR: refinement steps                       */
    int32_t check_every;   /* iterations launched between convergence checks */
    int32_t kernel_timing; /* k > 0: time the SpMV and block-Jacobi launches
                              of every k-th PCG iteration with HIP events
                              (sdsl_info; 1 = every iteration, 0 = off)     */
    int32_t border;        /* 1: with a low-rank term, the preconditioner
                              also eliminates its columns as a border:
                              (P + U C U^T)^{-1} through the k x k Schur
                              complement K = C^{-1} + U^T P^{-1} U (Sec. 2.1
                              bordered dense columns, Sec. 2.4 Schur coupling) */
    double refine_delta;   /* FP32_IR: residual reduction between refinement
                              points (0.1 typical)                           */
    int32_t refine_every;  /* FP32_IR: iterations after which a refinement
                              point is taken regardless of the reduction;
                              FP32_IR_RESTART: cap of one inner solve        */
    int32_t mc64;          /* 1: MC64 matching and scaling first (Sec. 3.3,
                              Alg. 3): the handle holds A' = Q Dr A Dc, whose
                              matched entries (largest diagonal product) sit
                              on the diagonal with magnitude 1 and no entry
                              is larger; filter, correction and factors are
                              built from A'; a solve takes b' = Q Dr b and
                              returns x = Dc y (relres and the tolerance are
                              those of A' y = b').  spd = 1: the matching of
                              an SPD matrix is the identity and the symmetric
                              scaling is 1 / sqrt(a_ii) (no permutation).
                              Block Jacobi without a low-rank term only; the
                              matrix must be readable on the host (a device
                              matrix is copied); refactor / update_values
                              take values of A and reuse the matching.
                              spmv, precond_apply and residual act on A'.    */
    sdsl_factor factor;    /* ILU0 (default) or COMPLETE                     */
    int32_t graphs;        /* 1: sdsl_solve issues the PCG iterations of each
                              check interval through the shared-launch kernels
                              with a one-handle table, recorded once as a HIP
                              graph and replayed (a launch per interval instead
                              of three per iteration); handles without a
                              low-rank term; results are bitwise those of
                              graphs = 0; kernel_timing does not time these
                              iterations                                      */
} sdsl_options;

typedef struct {
    int64_t nnz_kept;       /* entries of the filtered block preconditioner  */
    int64_t nnz_dropped;    /* in-block entries dropped by the filter        */
    int32_t pivot_fixes;    /* REPLACE policy: replaced pivots               */
    int32_t shifted_blocks; /* SHIFT policy: blocks refactored with a shift  */
    double max_shift;       /* SHIFT policy: largest relative shift used     */
    int32_t outer_iters;    /* FP32_IR refinement points of the last solve   */
    int32_t inner_iters;    /* Krylov iterations of the last solve (total)   */
    int32_t fp64_fallbacks; /* FP32 modes: FP64 solves of the residual eq.  */
    int32_t restarts;       /* restarts from the true residual               */
    double setup_ms;        /* last setup / refactor time                    */
    double solve_ms;        /* last solve time                               */
    double relres;          /* last true relative residual                   */
    int64_t bytes_per_iter; /* algorithmic bytes of one Krylov iteration     */
    int64_t device_bytes;   /* device memory held by the handle              */
    /* kernel_timing: summed durations and counts of the timed launches of
     * the last solve made before it converged (no-op launches after it are
     * excluded); index 0 = FP64 kernels, 1 = FP32 kernels */
    double spmv_ms[2];
    int64_t spmv_launches[2];
    double bj_ms[2];
    int64_t bj_launches[2];
    int64_t spmv_bytes[2];  /* algorithmic bytes of one SpMV launch          */
    int64_t bj_bytes[2];    /* algorithmic bytes of one fused PCG/BJ launch  */
    /* FP32 modes: the decisions of the last solve (at most SDSL_RF_HISTORY
     * are kept; rf_count counts them all).  Entry e: rf_it = iterations so
     * far, rf_nr = the true residual norm the decision was taken on,
     * rf_act = 0 done, 1 continue, 2 solve the residual equation in FP64
     * from the current solution, 3 revert to the last refinement point (or
     * discard the broken-down inner solve) and solve in FP64, 4 fail; rf_flag bit 0 = breakdown, bit 1 = a decision
     * after an FP64 solve of the residual equation.  rf_nb = ||b||.  The
     * rule is a tuned choice of this library (the paper states no
     * precision): a point is weak when its residual is above 0.5 times the
     * previous point's; 3 weak points in a row of the mixed recurrence, or 2
     * weak classical refinement steps, send the rest to FP64 solves of the
     * residual equation (fresh PCG to 0.5 of the remaining tolerance, at
     * most 4). */
    int32_t rf_count;
    int32_t rf_it[64];
    double rf_nr[64];
    int32_t rf_act[64];
    int32_t rf_flag[64];
    double rf_nb;
    int32_t mc64_moved;     /* MC64: rows matched to another column than their own */
    /* dependency levels of the triangular sweeps (forward + backward, summed
     * over a block's row chunks): the largest over the blocks and the mean */
    int32_t sweep_levels_max;
    double sweep_levels_mean;
} sdsl_info;
#define SDSL_RF_HISTORY 64

/* Fills *o with defaults: BJ, no filter, no correction, SHIFT(1e-2), SPD,
 * PCG, restart 30, max_iter 100000, FP64, inner_tol 1e-4, max_outer 30,
 * check_every 16, kernel_timing 0, border 1, refine_delta 0.1,
 * refine_every 500, mc64 0, factor ILU0, graphs 0. */
void sdsl_default_options(sdsl_options* o);

/* Device-memory provider of a handle (PyTorch's caching allocator in the
 * Python binding).  alloc returns `bytes` of device memory of the current
 * device, usable on `hip_stream` (the handle's stream), or NULL when it
 * cannot; free returns a block that alloc gave, after the handle's stream has
 * finished using it.  `ctx` is passed through and must stay valid while the
 * handle lives.  Every device allocation of the handle (at setup, and the
 * GMRES basis at its first GMRES solve) goes through it; pinned host staging
 * buffers do not.  A NULL allocator, or alloc == NULL and free == NULL, uses
 * hipMalloc / hipFree. */
typedef struct {
    void* (*alloc)(size_t bytes, void* hip_stream, void* ctx);
    void (*free)(void* ptr, size_t bytes, void* hip_stream, void* ctx);
    void* ctx;
} sdsl_allocator;

/* Device bytes a handle for this problem will hold (for admission control),
 * the GMRES/GCR basis included when o->krylov is SDSL_GMRES or SDSL_GCR.  For SDSL_BBD the
 * tail factors depend on the pattern, so A->row_ptr and A->col must then be
 * readable host memory (A->mem = SDSL_MEM_HOST); otherwise only the sizes are
 * read.  Returns 0 on invalid arguments, including a BBD pattern that is not
 * in bordered block diagonal form. */
size_t sdsl_footprint_bytes(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o,
                            const sdsl_lowrank* lr);

/* Creates a handle: validates A and the partition, copies A (and the
 * low-rank term, may be NULL) into handle-owned device memory, builds and
 * factors the preconditioner (filter Eq. (filter), correction Eq. (diagcorr),
 * ILU(0) of every block in one launch; for BBD also the dense Schur
 * complement and its LU).  `al` (may be NULL) provides the handle's device
 * memory; `hip_stream` (a hipStream_t, NULL = default stream) orders every
 * later call of the handle.  The caller's arrays may be freed when the call
 * returns.  On error *out is NULL and everything allocated was returned. */
sdsl_status sdsl_setup(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o,
                       const sdsl_lowrank* lr, const sdsl_allocator* al, void* hip_stream,
                       sdsl_handle* out);

/* New values for the same pattern (Sec. 3.4: the symbolic analysis is kept
 * and only the numerical factorisation is redone): new_val (DEVICE, nnz doubles in
 * the CSR order given at setup) replaces the operator values, and the filter,
 * correction and factorisation are redone.  Stream-ordered; returns after the
 * factorisation finished. */
sdsl_status sdsl_refactor(sdsl_handle h, const double* new_val);

/* New operator values only; the preconditioner is kept (Sec. 3.4, the
 * aggressive mode that reuses the numerical factorisation). */
sdsl_status sdsl_update_values(sdsl_handle h, const double* new_val);

/* Solves M x = b to ||b - Mx||_2 <= tol ||b||_2 with x0 = 0.  b and x are
 * DEVICE arrays of n doubles (x is overwritten).  On return *iters holds the
 * Krylov iterations (inner iterations summed for FP32_IR) and *relres the
 * true relative residual recomputed in compensated FP64.  Returns
 * SDSL_E_NOT_CONVERGED (x = last iterate) or SDSL_E_BREAKDOWN on failure. */
sdsl_status sdsl_solve(sdsl_handle h, const double* b, double* x, double tol, int32_t* iters,
                       double* relres);

/* Iteration limit of the handle's later solves (Krylov iterations, inner
 * ones summed for FP32_IR); max_iter >= 1.  A driver that reuses a
 * preconditioner (Sec. 3.4) caps a reused solve with it so that convergence
 * degradation shows as SDSL_E_NOT_CONVERGED early.  SDSL_E_STATE while an
 * asynchronous solve runs on h. */
sdsl_status sdsl_set_max_iter(sdsl_handle h, int32_t max_iter);

/* Solves k independent systems, one per handle, with their launches
 * interleaved on the handles' streams so that they overlap on the device.
 * Each result equals that of sdsl_solve on the same handle.  iters/relres
 * are HOST arrays of k entries.  A handle may appear once per batch
 * (SDSL_E_STATE for a repeat).  Returns the first non-OK status. */
sdsl_status sdsl_solve_batch(int32_t k, const sdsl_handle* hs, const double* const* b,
                             double* const* x, double tol, int32_t* iters, double* relres);

/* Asynchronous form of sdsl_solve for serving loops that keep several
 * handles in flight.  sdsl_solve_begin starts the solve (same arguments and
 * semantics as sdsl_solve; b and x must stay valid until sdsl_solve_end).
 * sdsl_solve_step never waits for the device: while the handle's stream is
 * still running earlier launches it returns at once with *done = 0;
 * otherwise it takes the next step (reads the device state, launches the
 * next batch of iterations) and sets *done = 1 once the solve has finished.
 * sdsl_solve_end (only after *done = 1) returns the solve's status and its
 * iterations and true relative residual.  One running solve per handle:
 * while it is unfinished, every call that uses the handle's vectors or
 * factors (solve, solve_begin, solve_batch, refactor, update_values,
 * set_max_iter, spmv, precond_apply, residual) returns SDSL_E_STATE.  The
 * result equals that of sdsl_solve. */
sdsl_status sdsl_solve_begin(sdsl_handle h, const double* b, double* x, double tol);
sdsl_status sdsl_solve_step(sdsl_handle h, int32_t* done);
sdsl_status sdsl_solve_end(sdsl_handle h, int32_t* iters, double* relres);

/* ---- shared launches for served solves --------------------------------
 * A group advances the running solves of several handles on ONE stream with
 * shared launches: each PCG iteration of all of them is one SpMV launch, one
 * block-Jacobi launch and one p-update launch, whose workgroups are the
 * handles' own grids laid end to end (per precision form and SpMV lane
 * count), so that small solves fill the device together.  Every handle's
 * workgroups compute exactly what its own launches compute, so each result
 * is bitwise the one sdsl_solve gives on the same handle.  Applies to PCG
 * iterations (FP64 and both FP32 modes) of handles without a low-rank term;
 * everything else a solve does (true residuals, refinement points, the
 * GMRES/BiCGSTAB/GCR methods, low-rank handles) runs as in sdsl_solve_step.
 *
 * sdsl_group_create: hip_stream is the stream every member handle was set up
 * on (NULL: the default stream); use_graphs = 1 records the iterations of
 * each shape of a step (member set, counts, grids) once as a HIP graph and
 * replays it (the kernels read the member table from device memory, so a
 * replay needs only the table copy); al as for sdsl_setup (NULL: hipMalloc)
 * provides the table.  The group keeps a device table, pinned staging and
 * up to 16 graphs until sdsl_group_destroy.
 * sdsl_group_begin: as sdsl_solve_begin, but the first iterations wait for
 * the group's next step, where they share its launches.
 * sdsl_group_step: for each of the k handles (HOST array, each at most once,
 * each with a solve begun by sdsl_solve_begin or sdsl_group_begin on this
 * group's stream): waits for its last iterations, takes its next step, and
 * sets done[i] = 1 once its solve has finished (then call sdsl_solve_end);
 * then launches every collected iteration.  Handles whose solve finished
 * are skipped.  SDSL_E_INVALID for a handle on another stream, SDSL_E_STATE
 * for one without a running solve; the other handles still advance, and the
 * first non-OK status is returned.  A handle must not be destroyed while its
 * solve runs.  Calls on one group must not overlap. */
typedef struct sdsl_group_s* sdsl_group;
typedef struct {
    int64_t flushes;         /* shared issues (one per step and kernel form)    */
    int64_t slot_issues;     /* handle issues they merged                        */
    int64_t launches;        /* kernel launches they made (3 per iteration)      */
    int64_t graph_launches;  /* issues replayed from a graph                     */
    int64_t captures;        /* graphs recorded                                  */
} sdsl_group_stats;
sdsl_status sdsl_group_create(void* hip_stream, int32_t use_graphs, const sdsl_allocator* al, sdsl_group* out);
sdsl_status sdsl_group_begin(sdsl_group g, sdsl_handle h, const double* b, double* x, double tol);
sdsl_status sdsl_group_step(sdsl_group g, int32_t k, const sdsl_handle* hs, int32_t* done);
sdsl_status sdsl_group_get_stats(sdsl_group g, sdsl_group_stats* out);
void sdsl_group_destroy(sdsl_group g);

sdsl_status sdsl_get_info(sdsl_handle h, sdsl_info* out);

/* Last error message of h (or of the calling thread when h is NULL). */
const char* sdsl_last_error(sdsl_handle h);

void sdsl_destroy(sdsl_handle h);

/* ---- single-step entry points (kernel-level checks) -------------------- */

/* y = M x (+ U diag(c) U^T x).  prec: SDSL_FP64 uses the FP64 values and
 * vectors; SDSL_FP32_IR uses the FP32 values with FP32 x and y (x, y point to
 * n floats).  DEVICE arrays; stream-ordered, returns after completion. */
sdsl_status sdsl_spmv(sdsl_handle h, int32_t prec, const void* x, void* y);

/* z = P^{-1} r with the handle's preconditioner (BJ: forward then backward
 * substitution per block, Sec. 2.3; BBD: the Schur-coupled solve, Sec. 2.4).
 * prec as for sdsl_spmv.  DEVICE arrays. */
sdsl_status sdsl_precond_apply(sdsl_handle h, int32_t prec, const void* r, void* z);

/* r = b - M x in compensated FP64; *norm receives ||r||_2.  DEVICE arrays. */
sdsl_status sdsl_residual(sdsl_handle h, const double* b, const double* x, double* r, double* norm);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): sdsl_residual computed
 * with no allocation at all.  Same arguments, results and errors as
 * sdsl_residual (r = b - M x in compensated FP64, *norm = ||r||_2); the
 * reduction partials live in a 128 KiB scratch array of the library, one per
 * device for the life of the process, instead of the handle's buffers.
 * Limit: 1 + (SpMV workgroups) + 2 k 32 doubles for a low-rank term of k
 * columns must fit 16384, which holds up to about 8M rows; larger systems get
 * SDSL_E_INVALID with the sizes in sdsl_last_error.  Every call on one
 * device shares that array, which keeps the last call's contents: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  The handle's device must be the current one. */
sdsl_status sdsl_residual_noalloc(sdsl_handle h, const double* b, const double* x, double* r, double* norm);

/* Copies the filtered preconditioner pattern and its factors to HOST arrays
 * (any pointer may be NULL): row_ptr[n_int+1] (int64), col[nnz_kept],
 * corrected[nnz_kept] (filtered + corrected values before factorisation),
 * lu[nnz_kept] (ILU(0) factors in place: strict lower = L, rest = U),
 * shifts[nblocks] (relative shift used per block). */
sdsl_status sdsl_get_factors(sdsl_handle h, int64_t* row_ptr, int32_t* col, double* corrected,
                             double* lu, double* shifts);

/* MC64 data of a handle set up with mc64 = 1 (HOST arrays of n entries):
 * row_of[k] = the row of A at row k of A' (Q), row_scale = dr (per row of
 * A), col_scale = dc (per column).  Any pointer may be NULL.  SDSL_E_STATE
 * when the handle has no MC64 transform. */
sdsl_status sdsl_get_mc64(sdsl_handle h, int32_t* row_of, double* row_scale, double* col_scale);

/* BBD only (Sec. 2.4): copies the dense border Schur complement's LU
 * factors with partial pivoting (row-major n_border x n_border, strict
 * lower = unit L, rest = U, after the row swaps), the pivot rows (piv[k] =
 * row swapped with row k at step k, 0-based) and its inverse (row-major) to
 * HOST arrays; any pointer may be NULL.  SDSL_E_STATE for a BJ handle. */
sdsl_status sdsl_get_schur(sdsl_handle h, double* lu, int32_t* piv, double* inv);

#ifdef __cplusplus
}
#endif
#endif /* SDSL_H */
