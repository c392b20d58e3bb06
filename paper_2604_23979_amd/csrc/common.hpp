// Internal declarations shared by the gfx950 kernels and the host runtime.
// Every kernel is hand-written HIP for CDNA4 (64-wide wavefronts).  The files
// are compiled with -ffp-contract=off: every fused multiply-add is written as
// fma(), so the arithmetic is exactly what the source says.
#pragma once
#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdsl.h"

namespace sdsl {

constexpr int kWave = 64;

// -------------------------------------------------------------- device state
// Per-solve scalars that the iteration kernels read and write on the device,
// so that no Krylov scalar round-trips through the host.
struct KrylovState {
    int done;        // set once converged / broken down: later kernels exit at entry
    int conv;        // 1: recurrence residual met the tolerance
    int breakdown;   // 1: (p, Mp) <= 0 or a non-finite scalar
    int iters;       // iteration count at the moment `done` was set
    int spin_err;    // a bounded in-workgroup wait gave up (never expected)
    int update;      // 1: a refinement point is due (residual fell below delta
                     //    times its last refined value, or refine_every passed)
    int it_refine;   // iteration index of the last refinement point
    int refine_every;
    double bb;       // ||b||^2 of the current (inner) right-hand side
    double tol2;     // tol^2 for the squared-residual test
    double rr0;      // ||r||^2 at the last refinement point
    double delta2;   // refinement trigger (0: never)
    double rzs[2];   // (r, z) of the last two iterations, parity-indexed
    // BiCGSTAB scalars of the last two iterations, parity-indexed
    double bi_rho[2];
    double bi_alpha[2];
    double bi_omega[2];
};

// -------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over aligned groups of G lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Deterministic block sum: per-wave shuffle tree, then wave 0 sums the wave
// results in wave order.  `scratch` holds >= blockDim.x / 64 doubles.  The
// result is valid in every thread.  Must be reached by all threads.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (l == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    if (w == 0) {
        s = (l < nw) ? scratch[l] : 0.0;
        s = wave_sum(s);
        if (l == 0) scratch[0] = s;
    }
    __syncthreads();
    s = scratch[0];
    __syncthreads();
    return s;
}

// Sum of a[0..m) in a fixed order (strided per thread, then block_sum), the
// same in every workgroup that calls it.
__device__ __forceinline__ double block_sum_array(const double* a, int m, double* scratch) {
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) s += a[i];
    return block_sum(s, scratch);
}

// -------------------------------------------------------------- sentinels
// A solution slot that is not yet written holds a signalling-NaN pattern
// that no arithmetic produces (arithmetic NaNs are quiet), so the value
// itself says whether it is ready.
template <typename T> struct Sentinel;
template <> struct Sentinel<double> {
    using Bits = unsigned long long;
    static constexpr Bits bits = 0x7FF40000DEADBEEFull;
};
template <> struct Sentinel<float> {
    using Bits = unsigned int;
    static constexpr Bits bits = 0x7FA0BEEFu;
};

// -------------------------------------------------------------- launchers
// Setup kernels (kernels_setup.hip).
struct ValidateOut {
    int bad_rows;        // rows with unsorted/duplicate/out-of-range columns
    int missing_diag;    // rows without a stored diagonal
    int nonfinite;       // non-finite values
    int bad_rowptr;      // decreasing row pointers
    int first_bad;       // smallest offending row (or INT_MAX)
};

void launch_validate(int n, const int64_t* rp64, const int* ci, const double* v, ValidateOut* out,
                     hipStream_t s);
void launch_count_nonfinite(int64_t m, const double* v, ValidateOut* out, hipStream_t s);
void launch_rowptr32(int n, const int64_t* rp64, int* rp32, hipStream_t s);
void launch_cast_f32(int64_t m, const double* a, float* b, hipStream_t s);
void launch_diag(int n, const int* rp, const int* ci, const double* v, double* diag, hipStream_t s);
void launch_filter_count(int n_int, const int* rp, const int* ci, const double* v, const double* diag,
                         const int* bp, int nblocks, int mode, double tau, int* cnt, double* dropsum,
                         hipStream_t s);
// exclusive scan of cnt[0..n) into out[0..n] (out[n] = total); tmp holds
// >= (n + 1023) / 1024 + 1 ints
void launch_scan(int n, const int* cnt, int* out, int* tmp, hipStream_t s);
void launch_filter_compact(int n_int, const int* rp, const int* ci, const double* v, const double* diag,
                           const int* bp, int nblocks, int mode, double tau, unsigned flags,
                           double delta, const double* dropsum, const int* prp, int* pci,
                           double* pv_corr, int* pdiag, hipStream_t s);
// split the in-place factors into L (strict lower) and U (strict upper +
// diagonal) arrays; lrp/urp must hold the exclusive scans of the counts
void launch_lu_counts(int n_int, const int* prp, const int* pdiag, int* lcnt, int* ucnt, hipStream_t s);
void launch_lu_split(int n_int, const int* prp, const int* pci, const double* pv, const int* pdiag, const int* lrp,
                     int* lci, double* lval, const int* urp, int* uci, double* uval, double* udiag, hipStream_t s);
void launch_ilu0(int nblocks, const int* bp, const int* prp, const int* pci, const double* pv_corr,
                 double* pv, const int* pdiag, int spd, int policy, double shift0, double* shifts,
                 int* nfix, int* block_status, int* spin_err, hipStream_t s);

// Iteration kernels (kernels_iter.hip).
struct CsrView {
    int n;
    const int* rp;
    const int* ci;
    int halo = 0;  // SpMV near window: rows of a workgroup +- halo columns staged in LDS (0: none)
};

struct LowRankDev {
    int k = 0;          // number of columns (0: none)
    int slices = 0;     // partial sums per column in the U^T x reduction
    const int* urp = nullptr;  // CSR n x k
    const int* uci = nullptr;
    const void* uv = nullptr;  // double or float
    const int* ucp = nullptr;  // CSC (k columns)
    const int* uri = nullptr;
    const void* ucv = nullptr;
    const void* c = nullptr;   // k scaling factors (same type as values)
    double* part = nullptr;    // [k * slices] (FP64 sums; compensated: 2x)
    double* fold = nullptr;    // [2 * kMaxRank] folded coefficients (see LrFold)
    unsigned* counter = nullptr;  // arrival count of the folding reduction (self-resetting)
};

// LR_SCALED: the last workgroup of a U^T x reduction leaves
// fold[j] = c_j (U^T x)_j (the operator's low-rank term) in fold[];
// LR_BORDER: only the slice partials, which the next kernel (the direction
// update, the border correction) folds into t = U^T x and K^{-1} t itself,
// so that the reduction needs no arrival count and no device-wide fence.
enum LrFold { LR_NONE = 0, LR_SCALED = 1, LR_BORDER = 2 };
constexpr int kMaxRank = 64;

int spmv_rows(int n, int grid);
int spmv_grid(int n);
void launch_spmv_near(int n, int grid, const int* rp, const int* ci, int halo, unsigned long long* count,
                      hipStream_t s);
constexpr int kSpmvThreads = 1024;
constexpr int kSpmvRows = 256;      // rows per SpMV workgroup for small systems
constexpr int kSpmvMaxRows = 1024;  // at most 16 waves x 64 rows
constexpr int kSpmvHalo = 2176;  // near-window halo (FP64 window: 36-43 KB of LDS)
int spmv_lanes(double mean_row);

template <typename T>
void launch_lowrank_tdot(const LowRankDev& lr, const T* x, const KrylovState* st, int fold, hipStream_t s);
template <typename V, typename F>
void launch_spmv(const CsrView& A, const F* v, const LowRankDev& lr, const V* x, V* y, double* part_dot,
                 const KrylovState* st, int lanes, int grid, hipStream_t s);
void launch_residual(const CsrView& A, const double* v, const LowRankDev& lr, const double* b,
                     const double* x, double* r, double* part, int lanes, int grid, hipStream_t s);
// ||a||^2 and similar final reductions into out[0] (one workgroup)
void launch_sum_partials(const double* part, int m, double* out, hipStream_t s);

// Block factors split for the sweeps: strict lower part (unit L) and strict
// upper part of U in CSR, and the diagonal of U; values double or float.
struct BJDev {
    int nblocks;
    const int* bp;
    const int* lrp;
    const int* lci;
    const void* lval;
    const int* urp;
    const int* uci;
    const void* uval;
    const void* udiag;
    const int2* lch;  // forward chunk table (k_bj_chunks layout)
    const int2* uch;  // backward chunk table
    const int* llev;  // per-row level inside its forward chunk
    const int* ulev;  // per-row level inside its backward chunk
    const int* lnl;   // levels per forward chunk (chunk-table indexing)
    const int* unl;   // levels per backward chunk
    const int* lell_c;   // chunk-interleaved newest entries of L rows (k_bj_ell)
    const void* lell_v;  // their values (factor type)
    const int* uell_c;   // the same for U rows
    const void* uell_v;
    const int* lorp;     // older entries of L rows (all but the newest kBjEllWidth): CSR
    const int* loci;
    const void* lov;     // their values (factor type)
    const int* uorp;     // the same for U rows
    const int* uoci;
    const void* uov;
    const int2* lperm;   // {row, entries} solved by each thread of a forward chunk (ELL group, then level order)
    const int2* uperm;   // the same for backward chunks
};

// MODE 0: z = P^{-1} r.  MODE 1: PCG step (alpha from partials, x/r update,
// ||r||^2 partial, z = P^{-1} r, (r,z) partial).  MODE 2: z = P^{-1} r and
// (r,z) partial (PCG start).  MODE 3: y = L^{-1} r only.  MODE 4:
// z = U^{-1} y only (y given).
struct PcgVecs {
    void* x;
    void* r;
    const void* p;
    const void* q;
    void* z;
    void* y;               // scratch for the forward-substitution result
    const double* part_pq; // SpMV partials of (p, q)
    int npq;
    double* part_rz;       // [2 * nblocks], parity-indexed
    double* part_rr;       // [nblocks]
};

// Border correction of a low-rank term in the preconditioner:
// z <- z - W s with s = Kinv t, t = U^T z (partials of the U^T x kernel).
struct BorderDev {
    int k = 0;                  // 0: no border
    int slices = 0;
    const double* part = nullptr;  // slice partials of U^T z (LR_BORDER), [k * slices]
    const double* W = nullptr;     // n x k, column-major
    const double* Kinv = nullptr;  // k x k, row-major
    // U^T p of the new direction without a pass over U: U^T z' = t - G s
    // with G = U^T W, so U^T p = t - G s + beta U^T p_old (FP64 vectors
    // only; up = nullptr: not kept).  ufold = c_j (U^T p)_j for the product.
    const double* G = nullptr;  // k x k, row-major
    const double* c = nullptr;  // k scales of the low-rank term
    double* up = nullptr;       // k: U^T p of the current direction
    double* ufold = nullptr;    // k: c_j (U^T p)_j
};

// ---------------------------------------------------------- shared launches
// Several handles' PCG iterations in one launch per kernel: each handle (a
// slot) keeps the workgroup grid, arguments and therefore the arithmetic of
// its own launches; a launch's workgroups are the slots' grids laid end to
// end (prefix sums in *_pre, ns + 1 entries, each slot's range starting at a
// multiple of 8 so that the XCD mapping of its workgroups is unchanged).
// The iteration index of slot s at offset k of a shared issue is it0 + k.
struct SpmvSlot {
    int n, halo, rows, grid;
    const int* rp;
    const int* ci;
    const void* v;
    const void* x;
    void* y;
    double* part_dot;
    const KrylovState* st;
};
struct BjSlot {
    BJDev P;
    PcgVecs Vv;
    KrylovState* st;
    int it0;
};
struct PupdSlot {
    int n, nb, grid, it0;
    void* p;
    const void* z;
    const double* part_rz;
    const double* part_rr;
    KrylovState* st;
};
struct SlotTable {
    const int* spmv_pre;
    const SpmvSlot* spmv;
    const int* bj_pre;
    const BjSlot* bj;
    const int* pu_pre;
    const PupdSlot* pu;
};
// One PCG iteration (SpMV with the (p, q) partials, block-Jacobi apply with
// the r/x update, p update) of the first ns slots at offset k; wg[3] = the
// workgroup totals of the three launches, shm = the largest SpMV window.
template <typename V, typename F>
void launch_slots_iteration(const SlotTable& t, int ns, int k, int lanes, const int* wg, size_t shm, hipStream_t s);
int pupdate_grid(int n);
// MC64 transform (Alg. 3): A' values, b' = Q Dr b, x = Dc y
void launch_mc64_values(int64_t nnz, const int* emap, const double* escale, const double* a, double* out,
                        hipStream_t s);
void launch_mc64_rhs(int n, const int* rowof, const double* rs, const double* b, double* out, hipStream_t s);
void launch_mc64_sol(int n, const double* cs, const double* y, double* x, hipStream_t s);
// host: maximum-product matching (row i -> column match[i]) and the scalings
// dr, dc from its duals; false when no matching uses nonzeros only
bool mc64_match(int n, const int64_t* rp, const int* ci, const double* v, std::vector<int>& match,
                std::vector<double>& dr, std::vector<double>& dc);

// pupdate modes
enum { PUPD_STEP = 0, PUPD_START = 1, PUPD_REAPPLY = 2 };
template <typename V, typename F>
void launch_bj(int mode, const BJDev& P, const PcgVecs& v, KrylovState* st, int it, hipStream_t s);
constexpr int kMaxBasisHost = 64;  // GMRES basis columns handled per multi-dot call
void launch_multidot(int n, int k, const double* V, int64_t ldv, const double* w, double* part, double* out,
                     double* acc, hipStream_t s);
void launch_multiaxpy(int n, int k, const double* V, int64_t ldv, const double* coef, double alpha, double* w,
                      double* nrm_part, hipStream_t s);
void launch_scale_inv_norm(int n, const double* nrm2, const double* w, double* v, hipStream_t s);
// BBD tail data (one entry per interior block b; offsets into the packed
// dense arrays): H_b = L_TT^{-1} E_T (t x ne, row-major), Gt_b (t x nf,
// row-major) = (F U_TT^{-1})^T, ecols/frows the border columns/rows of E/F.
struct TailDev {
    const int* bp = nullptr;       // block boundaries (device)
    const int* tail = nullptr;     // first tail row per block
    const int* ne = nullptr;       // border columns touched by E_b
    const int* nf = nullptr;       // border rows touched by F_b
    const int64_t* hoff = nullptr; // H_b offset
    const int64_t* goff = nullptr; // Gt_b offset
    const int* ecoff = nullptr;    // offset of block b's ecols
    const int* fvoff = nullptr;    // offset of block b's frows (and partials)
    const int* trow = nullptr;     // first global tail-row number of block b
    const int* ecols = nullptr;
    const int* frows = nullptr;
    double* H = nullptr;
    double* G = nullptr;
    int ntail = 0;                 // total tail rows
};
void launch_dgemm_sub(bool a_t, int M, int N, int K, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double* C, int64_t ldc, const int* rmap, const int* cmap, hipStream_t s);
void launch_lu_panel(int n, int k0, int w, double* S, int* piv, int* bad, hipStream_t s);
void launch_trsm_block(bool lower, int w, const double* T, int64_t ldt, int d0, double* X, int64_t ldx, int r0,
                       int c0, int c1, hipStream_t s);
void launch_perm_identity(int n, const int* o, double* Y, hipStream_t s);
void launch_scatter_from(int64_t m, const int64_t* pos, const int64_t* at, const double* v, double* Out,
                         hipStream_t s);
void launch_tail_solves(const TailDev& T, int nblocks, int max_ne, int max_nf, const int* lrp, const int* lci,
                        const double* lval, const int* urp, const int* uci, const double* uval,
                        const double* udiag, hipStream_t s);
void launch_bbd_mid(const TailDev& T, int nblocks, int max_nf, int nbd, const double* Sinv, const int* fptr,
                    const int* fidx, double* gpart, const double* rb, double* g, double* w, double* xb,
                    hipStream_t s);
constexpr int kLuPanel = 64;
constexpr int kLuSub = 16;    // columns factored by one workgroup inside a panel
void launch_bj_ell(int nblocks, const int* bp, const int* rp, const int* ci, const double* val, const int* pos,
                   bool fwd, int* ec, double* ev64, float* ev32, hipStream_t s);
constexpr int kBjThreads = 512;  // threads (and rows per chunk) of a triangular-sweep workgroup
constexpr int kBjEllWidth = 24;  // entries per row in the interleaved copies
void launch_bj_old(int n, const int* rp, const int* ci, const double* val, int* cnt, int* tmp, int* orp, int* oci,
                   double* ov64, float* ov32, hipStream_t s);
void launch_bj_chunks(int nblocks, const int* bp, const int* lrp, const int* urp, int2* lch, int2* uch,
                      hipStream_t s);
void launch_bj_levels(int nblocks, const int* bp, const int* lrp, const int* lci, const int* urp, const int* uci,
                      const int2* lch, const int2* uch, int* llev, int* ulev, int* lnl, int* unl, int2* lperm,
                      int2* uperm, int* lpos, int* upos, hipStream_t s);

template <typename T>
void launch_pcg_pupdate(int n, const PcgVecs& v, int nblocks, const BorderDev& bd, KrylovState* st, int it,
                        int mode, hipStream_t s);
// BiCGSTAB vector steps (kernels_iter.hip); partial arrays hold bicg_grid(n)
// entries
int bicg_grid(int n);
void launch_dot2(int n, const double* a, const double* b, const double* c, const double* d, double* pa, double* pc,
                 const KrylovState* st, hipStream_t s);
void launch_bicg_p(int n, const double* r, double* p, const double* v, const double* part_rho,
                   const double* part_rr, KrylovState* st, int it, bool first, hipStream_t s);
void launch_bicg_s(int n, const double* r, const double* v, double* sv, const double* part_rv, double* part_ss,
                   KrylovState* st, int it, hipStream_t s);
void launch_bicg_x(int n, double* x, const double* ph, const double* sh, const double* sv, const double* t, double* r,
                   const double* rh, const double* part_ss, const double* part_ts, const double* part_tt,
                   double* part_rho, double* part_rr, KrylovState* st, int it, hipStream_t s);
void launch_gcr_xr(int n, double* x, double* r, double* p, double* q, const double* nu2, const double* nu02,
                   const double* part_rq, double* part_rr, hipStream_t s);
template <typename T>
void launch_border_fix(int n, T* z, const BorderDev& bd, hipStream_t s);
// border setup: dense column j of U (CSC) into e; K = diag(1/c) + U^T W; Kinv
void launch_scatter_column(int n, const int* ucp, const int* uri, const double* ucv, int j, double* e,
                           hipStream_t s);
void launch_border_k(int n, int k, const int* ucp, const int* uri, const double* ucv, const double* c,
                     const double* W, double* K, double* G, hipStream_t s);
void launch_small_inverse(int k, const double* K, double* Kinv, int* status, hipStream_t s);

// vector helpers
template <typename T>
void launch_fill(int64_t n, T* a, T val, hipStream_t s);
template <typename T>
void launch_copy(int64_t n, const T* a, T* b, hipStream_t s);
void launch_sqnorm_partials(int n, const double* a, double* part, int grid, hipStream_t s);
void launch_ir_scale_cast(int n, const double* r, const double* nr, float* rs, hipStream_t s);
void launch_ir_update(int n, double* x, const double* nr, const float* d, hipStream_t s);
void launch_init_state(KrylovState* st, const double* part_bb, int m, double tol, double delta,
                       hipStream_t s);
// after a refinement point at iteration `it`: rr0 = sum(part), clear
// done/conv/update (keep rzs), next forced refinement after `every` more
void launch_refine_state(KrylovState* st, const double* part, int m, int it, int every, hipStream_t s);
void launch_sqnorm_f32_partials(int n, const float* a, double* part, int grid, hipStream_t s);

}  // namespace sdsl
