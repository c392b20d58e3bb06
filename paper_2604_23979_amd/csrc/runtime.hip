// Host runtime and C ABI of the solver: the handle, preconditioner setup and
// refactorisation, and the Krylov drivers (PCG in FP64; PCG over FP32
// operator values and factors inside FP64 refinement; classical FP32 inner
// refinement).  Every numerical step runs in the gfx950 kernels; the host only
// sequences launches and reads a few scalars.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <queue>
#include <vector>

#include "common.hpp"

using namespace sdsl;

namespace {

struct Error {
    sdsl_status st;
    std::string msg;
};

[[noreturn]] void fail(sdsl_status st, const std::string& m) { throw Error{st, m}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(SDSL_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

thread_local std::string g_thread_err;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// -------------------------------------------------------------------- handle
namespace {
struct SolveTask;
void delete_task(SolveTask* t);
}  // namespace
struct sdsl_group_s;
void delete_group(sdsl_group_s* g);

struct sdsl_group_s;

struct sdsl_ctx {
    hipStream_t s = nullptr;
    SolveTask* task = nullptr;  // solve started by sdsl_solve_begin
    sdsl_group_s* defer = nullptr;  // set while a group step collects this handle's iterations
    bool unflushed = false;         // iterations collected by a group and not yet launched
    sdsl_group_s* holder = nullptr; // the group holding them
    sdsl_group_s* own = nullptr;    // graphs = 1: the one-handle group of sdsl_solve
    sdsl_options o{};
    int n = 0, n_int = 0, nbd = 0, nb = 0;
    int64_t nnz = 0;
    std::vector<int> bp_h;
    std::vector<std::pair<void*, size_t>> allocs;
    size_t bytes = 0;
    sdsl_allocator al{};  // caller's device-memory provider (alloc == NULL: hipMalloc / hipFree)
    std::string err;

    // operator
    int *bp = nullptr, *rp = nullptr, *ci = nullptr;
    double* v = nullptr;
    float* v32 = nullptr;
    double* diag = nullptr;
    int lanes = 4, grid = 8;
    // low-rank term (kept in FP64 in every mode)
    LowRankDev lr{};
    int64_t lr_nnz = 0;
    // block-Jacobi preconditioner: filtered + corrected values, in-place
    // ILU(0) factors, and the split copies the sweeps read
    int *prp = nullptr, *pci = nullptr, *pdiag = nullptr, *cnt = nullptr, *scan_tmp = nullptr;
    double *pv_corr = nullptr, *pv = nullptr, *dropsum = nullptr, *shifts = nullptr;
    int *nfix = nullptr, *bstatus = nullptr, *spin_err = nullptr;
    int *lrp = nullptr, *lci = nullptr, *urp = nullptr, *uci = nullptr, *ucnt = nullptr;
    int2 *lch = nullptr, *uch = nullptr;  // sweep chunk tables
    int halo = 0;                          // SpMV near-window halo (0: gather from memory)
    int *lnl = nullptr, *unl = nullptr, *llev = nullptr, *ulev = nullptr;  // chunk-local levels
    double *lval = nullptr, *uval = nullptr, *udiag = nullptr;
    float *lval32 = nullptr, *uval32 = nullptr, *udiag32 = nullptr;
    // chunk-interleaved newest entries of every factor row (the sweeps' copies)
    int *lell_c = nullptr, *uell_c = nullptr;
    double *lell_v = nullptr, *uell_v = nullptr;
    float *lell_v32 = nullptr, *uell_v32 = nullptr;
    // older entries of the longer factor rows (CSR per triangle)
    int *lorp = nullptr, *loci = nullptr, *uorp = nullptr, *uoci = nullptr;
    int2 *lperm = nullptr, *uperm = nullptr;  // row placement on the sweep threads
    int *lpos = nullptr, *upos = nullptr;
    double *lov = nullptr, *uov = nullptr;
    float *lov32 = nullptr, *uov32 = nullptr;
    int p_nnz = 0;
    int64_t pcap = 0;  // capacity of the filtered / factor entry arrays
    // border correction of the low-rank term (W = P^{-1} U, K^{-1})
    double* W64 = nullptr;
    double *Kmat = nullptr, *Kinv = nullptr, *Gmat = nullptr, *lr_up = nullptr, *lr_ufold = nullptr;
    int* kstat = nullptr;
    BorderDev bd{};
    // Krylov workspace
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *d = nullptr, *rf = nullptr;
    double* xref = nullptr;  // mixed mode: the solution at the last refinement point
    double* y = nullptr;     // forward-sweep scratch of the FP64 solve
    float* y32 = nullptr;    // forward-sweep scratch of FP32 solves
    float *x32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr;
    double *part_pq = nullptr, *part_rz = nullptr, *part_rr = nullptr, *part_b = nullptr, *part_res = nullptr;
    double* bi_part = nullptr;  // BiCGSTAB partials: 6 arrays of bicg_grid(n)
    double* scal = nullptr;  // [0] = ||r||^2 of the latest true residual, [1] = ||b||^2
    KrylovState* st = nullptr;
    KrylovState* st_h = nullptr;  // pinned
    double* scal_h = nullptr;     // pinned
    ValidateOut* vout = nullptr;
    ValidateOut* vout_h = nullptr;
    sdsl_info info{};
    // kernel timing: three events per iteration (SpMV start, SpMV end = BJ
    // start, BJ end), reused across batches
    std::vector<hipEvent_t> ev;
    // GMRES workspace (allocated on the first GMRES solve): basis V
    // (m+1 columns of n), preconditioned basis Z (m columns), multi-dot
    // partials, device coefficient columns, pinned host staging
    int gm_cap = 0;
    // BBD (Sec. 2.4): tails and dense tail factors, Schur LU and inverse
    bool bbd = false;
    TailDev tdev{};
    int bbd_max_ne = 0, bbd_max_nf = 0;
    std::vector<int> bbd_ne, bbd_nf, bbd_tail;
    std::vector<int64_t> bbd_hoff, bbd_goff;
    std::vector<int> bbd_ecoff, bbd_fvoff;
    int64_t bbd_nh = 0, bbd_ng = 0, bbd_nc = 0;   // COO lengths (H, Gt, C)
    int64_t *bbd_hpos = nullptr, *bbd_hat = nullptr, *bbd_gpos = nullptr, *bbd_gat = nullptr;
    int64_t *bbd_cpos = nullptr, *bbd_cat = nullptr;
    int *bbd_fptr = nullptr, *bbd_fidx = nullptr, *bbd_piv = nullptr, *bbd_ord = nullptr, *bbd_bad = nullptr;
    double *bbd_S = nullptr, *bbd_Sinv = nullptr, *bbd_gpart = nullptr, *bbd_g = nullptr;
    double *gV = nullptr, *gZ = nullptr, *gpart = nullptr, *gnrm = nullptr;
    double *ghcol = nullptr, *gh2 = nullptr, *gy = nullptr;
    double* gh_h = nullptr;  // pinned, kMaxBasisHost + 2 doubles
    // MC64 transform (Alg. 3): the handle holds A' = Q Dr A Dc
    bool mc64 = false;
    std::vector<int> m_rowof_h;          // row of A at each row of A'
    std::vector<double> m_dr_h, m_dc_h;  // dr per row of A, dc per column
    int *m_rowof = nullptr, *m_emap = nullptr;
    double *m_rs = nullptr, *m_cs = nullptr, *m_escale = nullptr, *m_b = nullptr, *m_y = nullptr;

    template <typename T>
    T* alloc(size_t count) {
        void* ptr = nullptr;
        const size_t b = std::max<size_t>(count, 1) * sizeof(T);
        if (al.alloc) {
            ptr = al.alloc(b, (void*)s, al.ctx);
        } else if (hipMalloc(&ptr, b) != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
        }
        if (!ptr) fail(SDSL_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
        allocs.push_back({ptr, b});
        bytes += b;
        return (T*)ptr;
    }
    void give_back(void* ptr, size_t b) {
        if (al.alloc) al.free(ptr, b, (void*)s, al.ctx);
        else (void)hipFree(ptr);
    }
    void release(void* ptr) {
        for (auto it = allocs.begin(); it != allocs.end(); ++it)
            if (it->first == ptr) {
                const size_t b = it->second;
                allocs.erase(it);
                give_back(ptr, b);
                bytes -= b;
                return;
            }
    }
    ~sdsl_ctx() {
        if (s) (void)hipStreamSynchronize(s);
        if (task) delete_task(task);
        if (own) delete_group(own);
        for (auto& a : allocs) give_back(a.first, a.second);
        if (st_h) (void)hipHostFree(st_h);
        if (scal_h) (void)hipHostFree(scal_h);
        if (vout_h) (void)hipHostFree(vout_h);
        if (gh_h) (void)hipHostFree(gh_h);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    void sync() { hip_check(hipStreamSynchronize(s), "stream synchronize"); }
    void check_launch() { hip_check(hipGetLastError(), "kernel launch"); }
};

namespace {

// ------------------------------------------------------------ setup helpers
void validate_values(sdsl_ctx* h, const int64_t* rp64_dev) {
    launch_validate(h->n, rp64_dev, h->ci, h->v, h->vout, h->s);
    h->check_launch();
    hip_check(hipMemcpyAsync(h->vout_h, h->vout, sizeof(ValidateOut), hipMemcpyDeviceToHost, h->s), "copy");
    h->sync();
    const ValidateOut& o = *h->vout_h;
    if (o.bad_rowptr) fail(SDSL_E_INVALID, "row_ptr decreases at row " + std::to_string(o.first_bad));
    if (o.bad_rows)
        fail(SDSL_E_INVALID, std::to_string(o.bad_rows) + " rows with unsorted, duplicate or out-of-range "
                                                          "columns (first row " + std::to_string(o.first_bad) + ")");
    if (o.missing_diag)
        fail(SDSL_E_INVALID, std::to_string(o.missing_diag) + " rows without a stored diagonal (first row " +
                                 std::to_string(o.first_bad) + ")");
    if (o.nonfinite) fail(SDSL_E_INVALID, "non-finite matrix values (first row " + std::to_string(o.first_bad) + ")");
}

// new operator values must be finite (same pattern, so nothing else changes)
// new operator values (device, in the order of A): copied, or mapped to A'
void take_values(sdsl_ctx* h, const double* vals) {
    if (h->mc64) launch_mc64_values(h->nnz, h->m_emap, h->m_escale, vals, h->v, h->s);
    else hip_check(hipMemcpyAsync(h->v, vals, h->nnz * sizeof(double), hipMemcpyDeviceToDevice, h->s), "copy");
    h->check_launch();
}

// Alg. 3 step 1 on the host: matching and scalings (or, for SPD, the
// identity with 1 / sqrt(a_ii)), then A' = Q Dr A Dc in CSR with, per entry
// of A, its position in A' and its factor dr_row dc_col; rs = dr of the row
// of A at each row of A'
void mc64_transform(const sdsl_csr* A, bool spd, sdsl_ctx* h, std::vector<int64_t>& rp2, std::vector<int>& ci2,
                    std::vector<double>& v2, std::vector<int>& emap, std::vector<double>& escale,
                    std::vector<double>& rs) {
    const int n = A->n;
    const int64_t nnz = A->nnz;
    if (nnz >= (int64_t(1) << 31)) fail(SDSL_E_INVALID, "MC64 limited to 2^31 entries");
    std::vector<int64_t> rp(n + 1);
    std::vector<int> ci(nnz);
    std::vector<double> v(nnz);
    const hipMemcpyKind k = A->mem == SDSL_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    if (!A->row_ptr || !A->col || !A->val) fail(SDSL_E_INVALID, "null CSR arrays");
    hip_check(hipMemcpy(rp.data(), A->row_ptr, (n + 1) * sizeof(int64_t), k), "copy");
    hip_check(hipMemcpy(ci.data(), A->col, nnz * sizeof(int), k), "copy");
    hip_check(hipMemcpy(v.data(), A->val, nnz * sizeof(double), k), "copy");
    if (rp[0] != 0 || rp[n] != nnz) fail(SDSL_E_INVALID, "row_ptr must run from 0 to nnz");
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) fail(SDSL_E_INVALID, "row_ptr must not decrease");
    for (int64_t q = 0; q < nnz; ++q) {
        if (ci[q] < 0 || ci[q] >= n) fail(SDSL_E_INVALID, "column index out of range");
        if (!std::isfinite(v[q])) fail(SDSL_E_INVALID, "non-finite matrix values");
    }
    std::vector<int> match;
    if (spd) {
        // |a_ij| <= sqrt(a_ii a_jj) makes the identity the best matching;
        // the symmetric scaling sqrt(dr dc) is then 1 / sqrt(a_ii)
        match.resize(n);
        h->m_dr_h.assign(n, 0.0);
        for (int i = 0; i < n; ++i) {
            match[i] = i;
            double d = 0.0;
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
                if (ci[q] == i) d = v[q];
            if (!(d > 0.0)) fail(SDSL_E_INVALID, "SPD mode needs a positive diagonal");
            h->m_dr_h[i] = 1.0 / std::sqrt(d);
        }
        h->m_dc_h = h->m_dr_h;
    } else if (!mc64_match(n, rp.data(), ci.data(), v.data(), match, h->m_dr_h, h->m_dc_h)) {
        fail(SDSL_E_STRUCTURE, "MC64: the matrix has no matching of nonzeros (structurally singular)");
    }
    h->mc64 = true;
    h->m_rowof_h.assign(n, 0);
    int moved = 0;
    for (int i = 0; i < n; ++i) {
        h->m_rowof_h[match[i]] = i;
        moved += match[i] != i;
    }
    h->info.mc64_moved = moved;
    rp2.assign(n + 1, 0);
    ci2.resize(nnz);
    v2.resize(nnz);
    emap.resize(nnz);
    escale.resize(nnz);
    rs.resize(n);
    for (int kk = 0; kk < n; ++kk) {
        const int r = h->m_rowof_h[kk];
        rs[kk] = h->m_dr_h[r];
        rp2[kk + 1] = rp2[kk] + (rp[r + 1] - rp[r]);
        int64_t out = rp2[kk];
        for (int64_t q = rp[r]; q < rp[r + 1]; ++q, ++out) {
            const double f = h->m_dr_h[r] * h->m_dc_h[ci[q]];
            ci2[out] = ci[q];
            v2[out] = f * v[q];
            emap[q] = (int)out;
            escale[q] = f;
        }
    }
}

void check_values(sdsl_ctx* h, const double* vals) {
    launch_count_nonfinite(h->nnz, vals, h->vout, h->s);
    h->check_launch();
    hip_check(hipMemcpyAsync(h->vout_h, h->vout, sizeof(ValidateOut), hipMemcpyDeviceToHost, h->s), "copy");
    h->sync();
    if (h->vout_h->nonfinite) fail(SDSL_E_INVALID, "non-finite matrix values");
}

BJDev bj_dev(sdsl_ctx* h, bool fp32) {
    BJDev P;
    P.nblocks = h->nb;
    P.bp = h->bp;
    P.lrp = h->lrp;
    P.lci = h->lci;
    P.urp = h->urp;
    P.uci = h->uci;
    P.lval = fp32 ? (const void*)h->lval32 : (const void*)h->lval;
    P.uval = fp32 ? (const void*)h->uval32 : (const void*)h->uval;
    P.udiag = fp32 ? (const void*)h->udiag32 : (const void*)h->udiag;
    P.lch = h->lch;
    P.uch = h->uch;
    P.llev = h->llev;
    P.ulev = h->ulev;
    P.lnl = h->lnl;
    P.unl = h->unl;
    P.lell_c = h->lell_c;
    P.uell_c = h->uell_c;
    P.lell_v = fp32 ? (const void*)h->lell_v32 : (const void*)h->lell_v;
    P.uell_v = fp32 ? (const void*)h->uell_v32 : (const void*)h->uell_v;
    P.lorp = h->lorp;
    P.loci = h->loci;
    P.lov = fp32 ? (const void*)h->lov32 : (const void*)h->lov;
    P.uorp = h->uorp;
    P.uoci = h->uoci;
    P.uov = fp32 ? (const void*)h->uov32 : (const void*)h->uov;
    P.lperm = h->lperm;
    P.uperm = h->uperm;
    return P;
}

// W = P^{-1} U column by column (block-Jacobi applies), K = C^{-1} + U^T W
// and its inverse; rebuilt with every factorisation.
void build_border(sdsl_ctx* h) {
    h->bd = BorderDev{};
    if (!h->o.border || h->lr.k <= 0) return;
    const int k = h->lr.k, n = h->n;
    if (!h->W64) {
        h->W64 = h->alloc<double>((size_t)k * n);
        h->Kmat = h->alloc<double>((size_t)k * k);
        h->Kinv = h->alloc<double>((size_t)k * k);
        h->Gmat = h->alloc<double>((size_t)k * k);
        h->lr_up = h->alloc<double>(k);
        h->lr_ufold = h->alloc<double>(kMaxRank);
        h->kstat = h->alloc<int>(1);
    }
    PcgVecs V{};
    for (int j = 0; j < k; ++j) {
        launch_scatter_column(n, h->lr.ucp, h->lr.uri, (const double*)h->lr.ucv, j, h->d, h->s);
        V.r = h->d;
        V.z = h->W64 + (size_t)j * n;
        V.y = h->y;
        launch_bj<double, double>(0, bj_dev(h, false), V, nullptr, 0, h->s);
    }
    launch_border_k(n, k, h->lr.ucp, h->lr.uri, (const double*)h->lr.ucv, (const double*)h->lr.c, h->W64, h->Kmat,
                    h->Gmat, h->s);
    launch_small_inverse(k, h->Kmat, h->Kinv, h->kstat, h->s);
    h->check_launch();
    int bad = 0;
    hip_check(hipMemcpyAsync(&bad, h->kstat, sizeof(int), hipMemcpyDeviceToHost, h->s), "copy");
    h->sync();
    if (bad) fail(SDSL_E_BREAKDOWN, "border Schur complement K = C^-1 + U^T P^-1 U is singular");
    h->bd = BorderDev{k, h->lr.slices, h->lr.part, h->W64, h->Kinv, h->Gmat, (const double*)h->lr.c, h->lr_up,
                      h->lr_ufold};
}

// ---------------------------------------------------------------- BBD
// Structure of the bordered block diagonal form (Sec. 2.4), from the host
// copy of the pattern: interior rows may couple only inside their block and
// to the border; a block's tail starts at the first row with a border
// column (E) or the first column referenced by a border row (F).  Per block
// the distinct border columns of E and rows of F, the dense tail factor
// layouts, and the positions of the E, F and C entries in the CSR (so that
// new values only need a gather).
struct BbdPattern {
    std::vector<int> tail;                     // first local row of each block's tail
    std::vector<std::vector<int>> ecols, frows;  // distinct border columns of E, rows of F
};
// The structure above from a validated host pattern (rows [0, n), interior
// rows [0, ni), blocks bp); the E columns and F rows of a block are sorted
// and distinct.  Returns the first interior row that couples to another
// block, or -1.
static int bbd_pattern(int n, int ni, const std::vector<int>& bp, const int64_t* rp, const int* ci,
                       BbdPattern& P) {
    const int nb = (int)bp.size() - 1;
    std::vector<int> blk(ni);
    for (int b = 0; b < nb; ++b)
        for (int i = bp[b]; i < bp[b + 1]; ++i) blk[i] = b;
    P.tail.assign(bp.begin() + 1, bp.end());
    for (int i = 0; i < ni; ++i) {
        const int b = blk[i];
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int j = ci[q];
            if (j >= ni) P.tail[b] = std::min(P.tail[b], i);
            else if (j < bp[b] || j >= bp[b + 1]) return i;
        }
    }
    for (int i = ni; i < n; ++i)
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
            if (ci[q] < ni) P.tail[blk[ci[q]]] = std::min(P.tail[blk[ci[q]]], ci[q]);
    P.ecols.assign(nb, {});
    P.frows.assign(nb, {});
    for (int i = 0; i < ni; ++i)
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
            if (ci[q] >= ni) P.ecols[blk[i]].push_back(ci[q] - ni);
    for (int i = ni; i < n; ++i)
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
            if (ci[q] < ni) P.frows[blk[ci[q]]].push_back(i - ni);
    for (int b = 0; b < nb; ++b) {
        std::sort(P.ecols[b].begin(), P.ecols[b].end());
        P.ecols[b].erase(std::unique(P.ecols[b].begin(), P.ecols[b].end()), P.ecols[b].end());
        std::sort(P.frows[b].begin(), P.frows[b].end());
        P.frows[b].erase(std::unique(P.frows[b].begin(), P.frows[b].end()), P.frows[b].end());
    }
    return -1;
}

void setup_bbd(sdsl_ctx* h, const std::vector<int64_t>& rp, const std::vector<int>& ci) {
    const int n = h->n, ni = h->n_int, nbd = h->nbd, nb = h->nb;
    const std::vector<int>& bp = h->bp_h;
    BbdPattern P;
    const int bad = bbd_pattern(n, ni, bp, rp.data(), ci.data(), P);
    if (bad >= 0) fail(SDSL_E_STRUCTURE, "interior row " + std::to_string(bad) + " couples to another block");
    std::vector<int>& tail = P.tail;
    std::vector<std::vector<int>>& ecols = P.ecols;
    std::vector<std::vector<int>>& frows = P.frows;
    h->bbd_ne.assign(nb, 0);
    h->bbd_nf.assign(nb, 0);
    h->bbd_hoff.assign(nb + 1, 0);
    h->bbd_goff.assign(nb + 1, 0);
    h->bbd_ecoff.assign(nb + 1, 0);
    h->bbd_fvoff.assign(nb + 1, 0);
    std::vector<int> trow(nb + 1, 0);
    std::vector<int> ecat, frcat;
    std::vector<int> epos(nbd, -1), fpos(nbd, -1);
    std::vector<std::vector<std::pair<int, int>>> fslots(nbd);  // border row -> (block, column)
    for (int b = 0; b < nb; ++b) {
        const int t = bp[b + 1] - tail[b];
        h->bbd_ne[b] = (int)ecols[b].size();
        h->bbd_nf[b] = (int)frows[b].size();
        h->bbd_hoff[b + 1] = h->bbd_hoff[b] + (int64_t)t * h->bbd_ne[b];
        h->bbd_goff[b + 1] = h->bbd_goff[b] + (int64_t)t * h->bbd_nf[b];
        h->bbd_ecoff[b + 1] = h->bbd_ecoff[b] + h->bbd_ne[b];
        h->bbd_fvoff[b + 1] = h->bbd_fvoff[b] + h->bbd_nf[b];
        trow[b + 1] = trow[b] + t;
        ecat.insert(ecat.end(), ecols[b].begin(), ecols[b].end());
        frcat.insert(frcat.end(), frows[b].begin(), frows[b].end());
        for (int c = 0; c < h->bbd_nf[b]; ++c) fslots[frows[b][c]].push_back({b, c});
        h->bbd_max_ne = std::max(h->bbd_max_ne, h->bbd_ne[b]);
        h->bbd_max_nf = std::max(h->bbd_max_nf, h->bbd_nf[b]);
    }
    h->bbd_tail = tail;
    // entry positions: H (E entries), Gt (F entries), C (border-border)
    std::vector<int64_t> hpos, hat, gpos, gat, cpos, cat;
    for (int b = 0; b < nb; ++b) {
        for (int c = 0; c < h->bbd_ne[b]; ++c) epos[ecols[b][c]] = c;
        for (int i = tail[b]; i < bp[b + 1]; ++i)
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
                if (ci[q] >= ni) {
                    hpos.push_back(q);
                    hat.push_back(h->bbd_hoff[b] + (int64_t)(i - tail[b]) * h->bbd_ne[b] + epos[ci[q] - ni]);
                }
        for (int c = 0; c < h->bbd_ne[b]; ++c) epos[ecols[b][c]] = -1;
    }
    for (int b = 0; b < nb; ++b) {
        for (int c = 0; c < h->bbd_nf[b]; ++c) fpos[frows[b][c]] = c;
        for (int i = ni; i < n; ++i) {
            if (fpos[i - ni] < 0) continue;
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
                const int j = ci[q];
                if (j >= bp[b] && j < bp[b + 1]) {
                    gpos.push_back(q);
                    gat.push_back(h->bbd_goff[b] + (int64_t)(j - tail[b]) * h->bbd_nf[b] + fpos[i - ni]);
                }
            }
        }
        for (int c = 0; c < h->bbd_nf[b]; ++c) fpos[frows[b][c]] = -1;
    }
    for (int i = ni; i < n; ++i)
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q)
            if (ci[q] >= ni) {
                cpos.push_back(q);
                cat.push_back((int64_t)(i - ni) * nbd + (ci[q] - ni));
            }
    std::vector<int> fptr(nbd + 1, 0), fidx;
    for (int f = 0; f < nbd; ++f) {
        for (auto& bc : fslots[f]) fidx.push_back(h->bbd_fvoff[bc.first] + bc.second);
        fptr[f + 1] = (int)fidx.size();
    }
    auto up64 = [&](const std::vector<int64_t>& v) {
        int64_t* d = h->alloc<int64_t>(v.size());
        if (!v.empty()) hip_check(hipMemcpy(d, v.data(), v.size() * 8, hipMemcpyHostToDevice), "copy");
        return d;
    };
    auto up32 = [&](const std::vector<int>& v) {
        int* d = h->alloc<int>(v.size());
        if (!v.empty()) hip_check(hipMemcpy(d, v.data(), v.size() * 4, hipMemcpyHostToDevice), "copy");
        return d;
    };
    h->bbd_nh = (int64_t)hpos.size();
    h->bbd_ng = (int64_t)gpos.size();
    h->bbd_nc = (int64_t)cpos.size();
    h->bbd_hpos = up64(hpos);
    h->bbd_hat = up64(hat);
    h->bbd_gpos = up64(gpos);
    h->bbd_gat = up64(gat);
    h->bbd_cpos = up64(cpos);
    h->bbd_cat = up64(cat);
    h->bbd_fptr = up32(fptr);
    h->bbd_fidx = up32(fidx);
    TailDev T;
    T.bp = h->bp;
    T.tail = up32(tail);
    T.ne = up32(h->bbd_ne);
    T.nf = up32(h->bbd_nf);
    T.hoff = up64(h->bbd_hoff);
    T.goff = up64(h->bbd_goff);
    T.ecoff = up32(h->bbd_ecoff);
    T.fvoff = up32(h->bbd_fvoff);
    T.trow = up32(trow);
    T.ecols = up32(ecat);
    T.frows = up32(frcat);
    T.H = h->alloc<double>(h->bbd_hoff[nb]);
    T.G = h->alloc<double>(h->bbd_goff[nb]);
    T.ntail = trow[nb];
    h->tdev = T;
    h->bbd_S = h->alloc<double>((size_t)nbd * nbd);
    h->bbd_Sinv = h->alloc<double>((size_t)nbd * nbd);
    h->bbd_piv = h->alloc<int>(nbd);
    h->bbd_ord = h->alloc<int>(nbd);
    h->bbd_bad = h->alloc<int>(1);
    h->bbd_gpart = h->alloc<double>(std::max(1, h->bbd_fvoff[nb]));
    h->bbd_g = h->alloc<double>(nbd);
    h->bbd = true;
}

// Schur complement S = C - sum_b Gt_b^T H_b (MFMA), its LU with partial
// pivoting (blocked: panel, triangular solve, MFMA trailing update) and its
// inverse U^{-1} L^{-1} P (MFMA updates); rebuilt with every factorisation.
void build_bbd(sdsl_ctx* h) {
    if (!h->bbd) return;
    hipStream_t s = h->s;
    const int nbd = h->nbd, nb = h->nb;
    TailDev& T = h->tdev;
    hip_check(hipMemsetAsync(T.H, 0, std::max<int64_t>(1, h->bbd_hoff[nb]) * 8, s), "memset");
    hip_check(hipMemsetAsync(T.G, 0, std::max<int64_t>(1, h->bbd_goff[nb]) * 8, s), "memset");
    hip_check(hipMemsetAsync(h->bbd_S, 0, (size_t)nbd * nbd * 8, s), "memset");
    hip_check(hipMemsetAsync(h->bbd_bad, 0, sizeof(int), s), "memset");
    launch_scatter_from(h->bbd_nh, h->bbd_hpos, h->bbd_hat, h->v, T.H, s);
    launch_scatter_from(h->bbd_ng, h->bbd_gpos, h->bbd_gat, h->v, T.G, s);
    launch_scatter_from(h->bbd_nc, h->bbd_cpos, h->bbd_cat, h->v, h->bbd_S, s);
    launch_tail_solves(T, nb, h->bbd_max_ne, h->bbd_max_nf, h->lrp, h->lci, h->lval, h->urp, h->uci, h->uval,
                       h->udiag, s);
    for (int b = 0; b < nb; ++b) {
        const int t = h->bp_h[b + 1] - h->bbd_tail[b];
        launch_dgemm_sub(true, h->bbd_nf[b], h->bbd_ne[b], t, T.G + h->bbd_goff[b], h->bbd_nf[b],
                         T.H + h->bbd_hoff[b], h->bbd_ne[b], h->bbd_S, nbd, T.frows + h->bbd_fvoff[b],
                         T.ecols + h->bbd_ecoff[b], s);
    }
    double* S = h->bbd_S;
    const int P = kLuPanel;
    for (int k0 = 0; k0 < nbd; k0 += P) {
        const int w = std::min(P, nbd - k0);
        // the block column [k0, k0 + w) in sub-panels of kLuSub columns: each
        // is factored by one workgroup, then the block's later columns get
        // its triangular solve and rank-kLuSub update on many workgroups
        for (int s0 = k0; s0 < k0 + w; s0 += kLuSub) {
            const int ws = std::min(kLuSub, k0 + w - s0);
            launch_lu_panel(nbd, s0, ws, S, h->bbd_piv, h->bbd_bad, s);
            if (s0 + ws < k0 + w) {
                launch_trsm_block(true, ws, S, nbd, s0, S, nbd, s0, s0 + ws, k0 + w, s);
                launch_dgemm_sub(false, nbd - s0 - ws, k0 + w - s0 - ws, ws, S + (int64_t)(s0 + ws) * nbd + s0, nbd,
                                 S + (int64_t)s0 * nbd + s0 + ws, nbd, S + (int64_t)(s0 + ws) * nbd + s0 + ws, nbd,
                                 nullptr, nullptr, s);
            }
        }
        if (k0 + w < nbd) {
            launch_trsm_block(true, w, S, nbd, k0, S, nbd, k0, k0 + w, nbd, s);
            const int m = nbd - k0 - w;
            launch_dgemm_sub(false, m, m, w, S + (int64_t)(k0 + w) * nbd + k0, nbd, S + (int64_t)k0 * nbd + k0 + w,
                             nbd, S + (int64_t)(k0 + w) * nbd + k0 + w, nbd, nullptr, nullptr, s);
        }
    }
    h->check_launch();
    int bad = 0;
    std::vector<int> piv(nbd);
    hip_check(hipMemcpyAsync(&bad, h->bbd_bad, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(piv.data(), h->bbd_piv, nbd * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    h->sync();
    if (bad) fail(SDSL_E_BREAKDOWN, "the border Schur complement is singular (zero pivot)");
    // inverse: Y = P I, Y = L^{-1} Y, Sinv = U^{-1} Y
    std::vector<int> ord(nbd);
    for (int i = 0; i < nbd; ++i) ord[i] = i;
    for (int kk = 0; kk < nbd; ++kk) std::swap(ord[kk], ord[piv[kk]]);
    hip_check(hipMemcpy(h->bbd_ord, ord.data(), nbd * sizeof(int), hipMemcpyHostToDevice), "copy");
    double* X = h->bbd_Sinv;
    launch_perm_identity(nbd, h->bbd_ord, X, s);
    for (int k0 = 0; k0 < nbd; k0 += P) {
        const int w = std::min(P, nbd - k0);
        launch_trsm_block(true, w, S, nbd, k0, X, nbd, k0, 0, nbd, s);
        if (k0 + w < nbd)
            launch_dgemm_sub(false, nbd - k0 - w, nbd, w, S + (int64_t)(k0 + w) * nbd + k0, nbd,
                             X + (int64_t)k0 * nbd, nbd, X + (int64_t)(k0 + w) * nbd, nbd, nullptr, nullptr, s);
    }
    for (int k0 = ((nbd - 1) / P) * P; k0 >= 0; k0 -= P) {
        const int w = std::min(P, nbd - k0);
        launch_trsm_block(false, w, S, nbd, k0, X, nbd, k0, 0, nbd, s);
        if (k0 > 0)
            launch_dgemm_sub(false, k0, nbd, w, S + k0, nbd, X + (int64_t)k0 * nbd, nbd, X, nbd, nullptr, nullptr,
                             s);
    }
    h->check_launch();
    h->sync();
}

// Symbolic fill of LU without pivoting, one block [lo, hi) of the filtered
// pattern (columns inside the block, sorted, diagonal present): row i's
// pattern is its own entries plus, for every k < i in it (taken in
// increasing order, fill included), the entries of row k's U part right of
// k.  Appends the rows to rp / ci (global row offsets in rp).
void lu_fill_block(int lo, int hi, const std::vector<int>& prp, const std::vector<int>& pci, std::vector<int64_t>& rp,
                   std::vector<int>& ci) {
    const int m = hi - lo;
    std::vector<std::vector<int>> upat(m);  // U part (columns > row) of processed rows, local indices
    std::vector<int> mark(m, -1);
    std::vector<int> row;
    std::priority_queue<int, std::vector<int>, std::greater<int>> lower;
    for (int i = 0; i < m; ++i) {
        row.clear();
        for (int q = prp[lo + i]; q < prp[lo + i + 1]; ++q) {
            const int c = pci[q] - lo;
            mark[c] = i;
            row.push_back(c);
            if (c < i) lower.push(c);
        }
        while (!lower.empty()) {
            const int k = lower.top();
            lower.pop();
            for (int c : upat[k])
                if (mark[c] != i) {
                    mark[c] = i;
                    row.push_back(c);
                    if (c < i) lower.push(c);
                }
        }
        std::sort(row.begin(), row.end());
        for (int c : row)
            if (c > i) upat[i].push_back(c);
        for (int c : row) ci.push_back(c + lo);
        rp.push_back((int64_t)ci.size());
    }
}

// COMPLETE factorisation: the filtered, corrected pattern grows by its
// symbolic fill (values 0 at the new positions) before the elimination
void complete_fill(sdsl_ctx* h) {
    const int ni = h->n_int;
    h->sync();
    std::vector<int> prp(ni + 1), pd(ni);
    hip_check(hipMemcpy(prp.data(), h->prp, (ni + 1) * sizeof(int), hipMemcpyDeviceToHost), "copy");
    const int kept = prp[ni];
    std::vector<int> pci(kept);
    std::vector<double> pv(kept);
    hip_check(hipMemcpy(pci.data(), h->pci, kept * sizeof(int), hipMemcpyDeviceToHost), "copy");
    hip_check(hipMemcpy(pv.data(), h->pv_corr, kept * sizeof(double), hipMemcpyDeviceToHost), "copy");
    std::vector<int64_t> rp{0};
    std::vector<int> ci;
    ci.reserve(kept);
    for (int b = 0; b < h->nb; ++b) lu_fill_block(h->bp_h[b], h->bp_h[b + 1], prp, pci, rp, ci);
    const int64_t F = rp[ni];
    if (F >= (int64_t(1) << 31)) fail(SDSL_E_NOMEM, "complete factor limited to 2^31 entries");
    std::vector<int> rp32(ni + 1);
    std::vector<double> v(F, 0.0);
    for (int i = 0; i < ni; ++i) {
        rp32[i] = (int)rp[i];
        int64_t q = prp[i];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (q < prp[i + 1] && pci[q] == ci[e]) v[e] = pv[q++];
            if (ci[e] == i) pd[i] = (int)e;
        }
    }
    rp32[ni] = (int)F;
    if (F > h->pcap) {
        // every array sized by the factor's entries grows (no launch reads them now)
        auto grow_i = [&](int*& a) { h->release(a); a = h->alloc<int>(F); };
        auto grow_d = [&](double*& a) { h->release(a); a = h->alloc<double>(F); };
        auto grow_f = [&](float*& a) { h->release(a); a = h->alloc<float>(F); };
        grow_i(h->pci); grow_i(h->lci); grow_i(h->uci); grow_i(h->loci); grow_i(h->uoci);
        grow_d(h->pv_corr); grow_d(h->pv); grow_d(h->lval); grow_d(h->uval); grow_d(h->lov); grow_d(h->uov);
        grow_f(h->lval32); grow_f(h->uval32); grow_f(h->lov32); grow_f(h->uov32);
        h->pcap = F;
    }
    hip_check(hipMemcpyAsync(h->prp, rp32.data(), (ni + 1) * sizeof(int), hipMemcpyHostToDevice, h->s), "copy");
    hip_check(hipMemcpyAsync(h->pci, ci.data(), F * sizeof(int), hipMemcpyHostToDevice, h->s), "copy");
    hip_check(hipMemcpyAsync(h->pv_corr, v.data(), F * sizeof(double), hipMemcpyHostToDevice, h->s), "copy");
    hip_check(hipMemcpyAsync(h->pdiag, pd.data(), ni * sizeof(int), hipMemcpyHostToDevice, h->s), "copy");
    h->sync();  // the host vectors go out of scope
}

void build_precond(sdsl_ctx* h) {
    const double t0 = now_ms();
    hipStream_t s = h->s;
    launch_diag(h->n, h->rp, h->ci, h->v, h->diag, s);
    const int mode = h->o.filter;
    launch_filter_count(h->n_int, h->rp, h->ci, h->v, h->diag, h->bp, h->nb, mode, h->o.tau, h->cnt, h->dropsum, s);
    launch_scan(h->n_int, h->cnt, h->prp, h->scan_tmp, s);
    launch_filter_compact(h->n_int, h->rp, h->ci, h->v, h->diag, h->bp, h->nb, mode, h->o.tau, h->o.diag_flags,
                          h->o.delta, h->dropsum, h->prp, h->pci, h->pv_corr, h->pdiag, s);
    if (h->o.factor == SDSL_FACT_COMPLETE) complete_fill(h);
    hip_check(hipMemsetAsync(h->nfix, 0, sizeof(int), s), "memset");
    hip_check(hipMemsetAsync(h->spin_err, 0, sizeof(int), s), "memset");
    launch_ilu0(h->nb, h->bp, h->prp, h->pci, h->pv_corr, h->pv, h->pdiag, h->o.spd, h->o.pivot, h->o.shift0,
                h->shifts, h->nfix, h->bstatus, h->spin_err, s);
    // split copies for the sweeps (and their FP32 roundings)
    launch_lu_counts(h->n_int, h->prp, h->pdiag, h->cnt, h->ucnt, s);
    launch_scan(h->n_int, h->cnt, h->lrp, h->scan_tmp, s);
    launch_scan(h->n_int, h->ucnt, h->urp, h->scan_tmp, s);
    launch_lu_split(h->n_int, h->prp, h->pci, h->pv, h->pdiag, h->lrp, h->lci, h->lval, h->urp, h->uci, h->uval,
                    h->udiag, s);
    launch_bj_chunks(h->nb, h->bp, h->lrp, h->urp, h->lch, h->uch, s);
    launch_bj_levels(h->nb, h->bp, h->lrp, h->lci, h->urp, h->uci, h->lch, h->uch, h->llev, h->ulev, h->lnl, h->unl,
                     h->lperm, h->uperm, h->lpos, h->upos, s);
    launch_bj_ell(h->nb, h->bp, h->lrp, h->lci, h->lval, h->lpos, true, h->lell_c, h->lell_v, h->lell_v32, s);
    launch_bj_ell(h->nb, h->bp, h->urp, h->uci, h->uval, h->upos, false, h->uell_c, h->uell_v, h->uell_v32, s);
    launch_bj_old(h->n_int, h->lrp, h->lci, h->lval, h->cnt, h->scan_tmp, h->lorp, h->loci, h->lov, h->lov32, s);
    launch_bj_old(h->n_int, h->urp, h->uci, h->uval, h->cnt, h->scan_tmp, h->uorp, h->uoci, h->uov, h->uov32, s);
    h->check_launch();
    int kept = 0, nfix = 0, spin = 0, nl = 0, nu = 0;
    hip_check(hipMemcpyAsync(&kept, h->prp + h->n_int, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(&nl, h->lrp + h->n_int, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(&nu, h->urp + h->n_int, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(&nfix, h->nfix, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(&spin, h->spin_err, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    std::vector<int> bst(h->nb);
    std::vector<double> sh(h->nb);
    hip_check(hipMemcpyAsync(bst.data(), h->bstatus, h->nb * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(sh.data(), h->shifts, h->nb * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    std::vector<int> lnl(h->n_int + h->nb), unl(h->n_int + h->nb);
    hip_check(hipMemcpyAsync(lnl.data(), h->lnl, lnl.size() * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(unl.data(), h->unl, unl.size() * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    h->sync();
    {
        // dependency depth of each block's two sweeps (chunk-table indexing)
        int64_t tot = 0;
        int mx = 0;
        for (int b = 0; b < h->nb; ++b) {
            const int lo = h->bp_h[b], hi = h->bp_h[b + 1];
            const int nch = (hi - lo + kBjThreads - 1) / kBjThreads;
            int lv = 0;
            for (int q = 0; q < nch; ++q) lv += lnl[lo + b + q] + unl[lo + b + q];
            tot += lv;
            mx = std::max(mx, lv);
        }
        h->info.sweep_levels_max = mx;
        h->info.sweep_levels_mean = h->nb > 0 ? (double)tot / h->nb : 0.0;
    }
    h->p_nnz = kept;
    launch_cast_f32(nl, h->lval, h->lval32, s);
    launch_cast_f32(nu, h->uval, h->uval32, s);
    launch_cast_f32(h->n_int, h->udiag, h->udiag32, s);
    h->check_launch();
    h->info.nnz_kept = kept;
    h->info.pivot_fixes = nfix;
    h->info.shifted_blocks = 0;
    h->info.max_shift = 0.0;
    for (int b = 0; b < h->nb; ++b) {
        if (sh[b] > 0) { h->info.shifted_blocks++; h->info.max_shift = std::max(h->info.max_shift, sh[b]); }
    }
    if (spin) fail(SDSL_E_DEVICE, "ILU(0) in-workgroup wait limit exceeded");
    for (int b = 0; b < h->nb; ++b)
        if (bst[b] != 0)
            fail(SDSL_E_BREAKDOWN, "ILU(0) breakdown in block " + std::to_string(b) + " (pivot policy " +
                                       std::to_string((int)h->o.pivot) + ")");
    h->sync();
    build_border(h);
    build_bbd(h);
    h->info.setup_ms = now_ms() - t0;
    // algorithmic bytes: every array a launch must touch, once.  Index 0: FP64
    // values and vectors; index 1: FP32 values/factors with FP64 vectors.
    const int64_t n = h->n, ni = h->n_int, off = (int64_t)kept - ni;
    for (int p = 0; p < 2; ++p) {
        const int64_t f = p ? 4 : 8;
        h->info.spmv_bytes[p] = (f + 4) * h->nnz + 4 * (n + 1) + 2 * 8 * n;
        if (h->lr_nnz > 0) h->info.spmv_bytes[p] += 12 * h->lr_nnz + 4 * (n + 1);
        h->info.bj_bytes[p] = (f + 4) * off + f * ni + 8 * (ni + 1) + 2 * f * n + 7 * 8 * n;
    }
    h->info.bytes_per_iter = h->info.spmv_bytes[0] + h->info.bj_bytes[0] + 3 * 8 * n;
}

void setup_lowrank(sdsl_ctx* h, const sdsl_lowrank* lr) {
    if (!lr || lr->k <= 0) return;
    const int k = lr->k, n = h->n;
    if (k > kMaxRank) fail(SDSL_E_INVALID, "low-rank term limited to 64 columns");
    const sdsl_csr& U = lr->U;
    if (U.n != n || U.nnz < 0 || !U.row_ptr || (U.nnz > 0 && (!U.col || !U.val)) || !lr->c)
        fail(SDSL_E_INVALID, "bad low-rank term");
    std::vector<int64_t> urp(n + 1);
    std::vector<int> uci(U.nnz);
    std::vector<double> uv(U.nnz), c(k);
    const hipMemcpyKind kind = U.mem == SDSL_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    hip_check(hipMemcpy(urp.data(), U.row_ptr, (n + 1) * sizeof(int64_t), kind), "copy");
    if (U.nnz) {
        hip_check(hipMemcpy(uci.data(), U.col, U.nnz * sizeof(int), kind), "copy");
        hip_check(hipMemcpy(uv.data(), U.val, U.nnz * sizeof(double), kind), "copy");
    }
    hip_check(hipMemcpy(c.data(), lr->c, k * sizeof(double), kind), "copy");
    if (urp[0] != 0 || urp[n] != U.nnz) fail(SDSL_E_INVALID, "low-rank row_ptr does not span nnz");
    for (int i = 0; i < n; ++i) {
        if (urp[i + 1] < urp[i]) fail(SDSL_E_INVALID, "low-rank row_ptr decreases");
        for (int64_t p = urp[i]; p < urp[i + 1]; ++p)
            if (uci[p] < 0 || uci[p] >= k || !std::isfinite(uv[p])) fail(SDSL_E_INVALID, "bad low-rank entry");
    }
    for (double cj : c)
        if (!std::isfinite(cj) || cj == 0.0) fail(SDSL_E_INVALID, "low-rank scales must be finite and non-zero");
    // CSC copy for U^T x
    std::vector<int> cp(k + 1, 0), ri(U.nnz);
    std::vector<double> cv(U.nnz);
    for (int64_t p = 0; p < U.nnz; ++p) cp[uci[p] + 1]++;
    for (int j = 0; j < k; ++j) cp[j + 1] += cp[j];
    std::vector<int> pos(cp.begin(), cp.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int64_t p = urp[i]; p < urp[i + 1]; ++p) {
            ri[pos[uci[p]]] = i;
            cv[pos[uci[p]]] = uv[p];
            pos[uci[p]]++;
        }
    std::vector<int> urp32(n + 1);
    for (int i = 0; i <= n; ++i) urp32[i] = (int)urp[i];
    const int64_t m = U.nnz;
    h->lr_nnz = m;
    int* d_urp = h->alloc<int>(n + 1);
    int* d_uci = h->alloc<int>(m);
    double* d_uv = h->alloc<double>(m);
    int* d_ucp = h->alloc<int>(k + 1);
    int* d_uri = h->alloc<int>(m);
    double* d_ucv = h->alloc<double>(m);
    double* d_c = h->alloc<double>(k);
    const int slices = 32;
    double* part = h->alloc<double>(2 * k * slices);
    double* fold = h->alloc<double>(2 * kMaxRank);
    unsigned* counter = h->alloc<unsigned>(1);
    hip_check(hipMemset(counter, 0, sizeof(unsigned)), "memset");
    hip_check(hipMemcpy(d_urp, urp32.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_uci, uci.data(), m * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_uv, uv.data(), m * sizeof(double), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_ucp, cp.data(), (k + 1) * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_uri, ri.data(), m * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_ucv, cv.data(), m * sizeof(double), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_c, c.data(), k * sizeof(double), hipMemcpyHostToDevice), "copy");
    LowRankDev L;
    L.k = k;
    L.slices = slices;
    L.urp = d_urp;
    L.uci = d_uci;
    L.uv = d_uv;
    L.ucp = d_ucp;
    L.uri = d_uri;
    L.ucv = d_ucv;
    L.c = d_c;
    L.part = part;
    L.fold = fold;
    L.counter = counter;
    h->lr = L;
}

// ------------------------------------------------------------- PCG engine
// One PCG recurrence on the device with vectors of type V and operator
// values / factors of type F.  `start` forms z = P^{-1} r and p = z for the
// residual in r; `issue` launches up to `count` iterations (kernels become
// no-ops once the device state says done); `reapply` resumes after a
// refinement point replaced r; `poll` synchronises and reads the state.
template <typename V, typename F>
struct Pcg {
    sdsl_ctx* h;
    V *x, *r, *z, *p, *q;
    F* y;
    const F* v;
    BJDev P;
    PcgVecs Vv;
    int it = 0;  // next iteration index
    int batch_start = 0, batch_count = 0;
    static constexpr int kPrec = sizeof(F) == 4 ? 1 : 0;

    void init() {
        P = bj_dev(h, sizeof(F) == 4);
        Vv.x = x; Vv.r = r; Vv.p = p; Vv.q = q; Vv.z = z; Vv.y = y;
        Vv.part_pq = h->part_pq;
        Vv.npq = h->grid;
        Vv.part_rz = h->part_rz;
        Vv.part_rr = h->part_rr;
    }
    void set_x(V* xx) { x = xx; Vv.x = xx; }
    // FP64 directions with a border keep U^T p by its recurrence (the p
    // update writes the product's coefficients): no U^T p pass per iteration
    bool lr_rec() const { return sizeof(V) == 8 && h->bd.k > 0 && h->bd.up; }
    BorderDev border() const {
        BorderDev B = h->bd;
        if (!lr_rec()) B.up = nullptr;
        return B;
    }
    LowRankDev spmv_lr() const {
        LowRankDev L = h->lr;
        if (lr_rec()) L.fold = h->bd.ufold;
        return L;
    }
    void precondition(int j, int mode) {
        launch_bj<V, F>(2, P, Vv, h->st, j, h->s);
        if (h->bd.k > 0) launch_lowrank_tdot<V>(h->lr, z, nullptr, LR_BORDER, h->s);
        launch_pcg_pupdate<V>(h->n, Vv, h->nb, border(), h->st, j, mode, h->s);
        if (h->lr.k > 0 && !lr_rec()) launch_lowrank_tdot<V>(h->lr, p, h->st, LR_SCALED, h->s);
        h->check_launch();
    }
    void start(int it0) {
        precondition(it0 - 1, PUPD_START);
        it = it0;
    }
    void reapply(int j) {
        precondition(j, PUPD_REAPPLY);
        it = j + 1;
    }
    // kernel timing: iterations whose index is a multiple of kernel_timing
    // get three events (SpMV start, SpMV end = BJ start, BJ end); sampled[k]
    // = the batch position of the k-th timed iteration
    std::vector<int> sampled;
    void issue(int count) {
        if (h->defer && h->lr.k == 0 && h->bd.k == 0) {
            defer_issue(count);
            return;
        }
        const CsrView A{h->n, h->rp, h->ci, h->halo};
        const int period = h->o.kernel_timing;
        const LowRankDev lr_s = spmv_lr();
        const BorderDev bd_ = border();
        const bool rec = lr_rec();
        batch_start = it;
        batch_count = count;
        sampled.clear();
        for (int k = 0; k < count; ++k, ++it) {
            const bool timed = period > 0 && it % period == 0;
            int e = 0;
            if (timed) {
                e = 3 * (int)sampled.size();
                if ((int)h->ev.size() < e + 3) {
                    const size_t old = h->ev.size();
                    h->ev.resize(e + 3);
                    for (size_t i = old; i < h->ev.size(); ++i) hip_check(hipEventCreate(&h->ev[i]), "event create");
                }
                sampled.push_back(k);
            }
            if (timed) hip_check(hipEventRecord(h->ev[e], h->s), "event record");
            launch_spmv<V, F>(A, v, lr_s, p, q, h->part_pq, h->st, h->lanes, h->grid, h->s);
            if (timed) hip_check(hipEventRecord(h->ev[e + 1], h->s), "event record");
            launch_bj<V, F>(1, P, Vv, h->st, it, h->s);
            if (timed) hip_check(hipEventRecord(h->ev[e + 2], h->s), "event record");
            if (h->bd.k > 0) launch_lowrank_tdot<V>(h->lr, z, h->st, LR_BORDER, h->s);
            launch_pcg_pupdate<V>(h->n, Vv, h->nb, bd_, h->st, it, PUPD_STEP, h->s);
            if (h->lr.k > 0 && !rec) launch_lowrank_tdot<V>(h->lr, p, h->st, LR_SCALED, h->s);
        }
        h->check_launch();
    }
    // the same iterations, collected for the shared launches of a group
    void defer_issue(int count);
    const KrylovState& poll() {
        hip_check(hipMemcpyAsync(h->st_h, h->st, sizeof(KrylovState), hipMemcpyDeviceToHost, h->s), "copy");
        h->sync();
        if (h->st_h->spin_err) fail(SDSL_E_DEVICE, "triangular solve met a term not yet solved at its level (stale level tables)");
        if (!sampled.empty()) {
            // only launches made before the state said done did work
            int live = batch_count;
            if (h->st_h->done) live = std::max(0, std::min(batch_count, h->st_h->iters - batch_start));
            for (size_t q = 0; q < sampled.size() && sampled[q] < live; ++q) {
                float a = 0.f, b = 0.f;
                hip_check(hipEventElapsedTime(&a, h->ev[3 * q], h->ev[3 * q + 1]), "event time");
                hip_check(hipEventElapsedTime(&b, h->ev[3 * q + 1], h->ev[3 * q + 2]), "event time");
                h->info.spmv_ms[kPrec] += a;
                h->info.bj_ms[kPrec] += b;
                h->info.spmv_launches[kPrec] += 1;
                h->info.bj_launches[kPrec] += 1;
            }
        }
        sampled.clear();
        batch_count = 0;
        return *h->st_h;
    }
};

}  // namespace

// ------------------------------------------------------- shared launches
// Iterations that handles on one stream asked for during a group step; the
// flush lays every handle's SpMV, block-Jacobi and p-update grids end to end
// in one launch per kernel (per vector/factor type and SpMV lane count), so
// small solves fill the device together and pay one launch per kernel.  Each
// handle's workgroups see the grid, arguments and iteration index of its own
// launch, so its arithmetic, and its result, are those of a solve alone.
struct IssueRec {
    sdsl_ctx* h;
    int type;   // 0: FP64 vectors and factors, 1: FP64 vectors / FP32 factors, 2: FP32
    int lanes;
    int count;
    size_t shm;
    SpmvSlot sp;
    BjSlot bj;
    PupdSlot pu;
};

struct sdsl_group_s {
    hipStream_t s = nullptr;
    hipStream_t cap = nullptr;  // capture stream of the iteration graphs (nothing runs on it)
    bool graphs = false;
    sdsl_allocator al{};
    std::vector<IssueRec> recs;
    char* dev = nullptr;
    size_t dev_cap = 0;
    char* stage = nullptr;  // pinned
    size_t stage_cap = 0;
    hipEvent_t copied = nullptr;  // the last table copy has read the staging buffer
    bool copy_pending = false;
    struct Graph {
        std::vector<int64_t> key;
        hipGraphExec_t exec;
        uint64_t used;
    };
    std::vector<Graph> cache;
    uint64_t tick = 0;
    sdsl_group_stats stats{};

    ~sdsl_group_s() {
        if (s) (void)hipStreamSynchronize(s);
        for (auto& g : cache) (void)hipGraphExecDestroy(g.exec);
        if (dev) {
            if (al.alloc) al.free(dev, dev_cap, (void*)s, al.ctx);
            else (void)hipFree(dev);
        }
        if (stage) (void)hipHostFree(stage);
        if (copied) (void)hipEventDestroy(copied);
        if (cap) (void)hipStreamDestroy(cap);
    }
    void drop_graphs() {
        for (auto& g : cache) (void)hipGraphExecDestroy(g.exec);
        cache.clear();
    }
    void reserve(size_t bytes) {
        if (copy_pending) {
            hip_check(hipEventSynchronize(copied), "event synchronize");
            copy_pending = false;
        }
        if (bytes > stage_cap) {
            if (stage) (void)hipHostFree(stage);
            stage = nullptr;
            const size_t c = std::max<size_t>(bytes, 64 << 10);
            hip_check(hipHostMalloc((void**)&stage, c, hipHostMallocDefault), "pinned alloc");
            stage_cap = c;
        }
        if (bytes > dev_cap) {
            // graphs hold table addresses: rebuilt on the new table
            hip_check(hipStreamSynchronize(s), "stream synchronize");
            drop_graphs();
            if (dev) {
                if (al.alloc) al.free(dev, dev_cap, (void*)s, al.ctx);
                else (void)hipFree(dev);
            }
            dev = nullptr;
            const size_t c = std::max<size_t>(bytes, 64 << 10);
            void* ptr = nullptr;
            if (al.alloc) ptr = al.alloc(c, (void*)s, al.ctx);
            else if (hipMalloc(&ptr, c) != hipSuccess) {
                (void)hipGetLastError();
                ptr = nullptr;
            }
            if (!ptr) fail(SDSL_E_NOMEM, "device allocation of the slot table failed");
            dev = (char*)ptr;
            dev_cap = c;
        }
    }
    static void launch(int type, const SlotTable& t, int ns, int k, int lanes, const int* wg, size_t shm,
                       hipStream_t st) {
        if (type == 0) launch_slots_iteration<double, double>(t, ns, k, lanes, wg, shm, st);
        else if (type == 1) launch_slots_iteration<double, float>(t, ns, k, lanes, wg, shm, st);
        else launch_slots_iteration<float, float>(t, ns, k, lanes, wg, shm, st);
    }
    void flush();
};

namespace {
template <typename V, typename F>
void Pcg<V, F>::defer_issue(int count) {
    IssueRec rec{};
    rec.h = h;
    rec.type = sizeof(V) == 4 ? 2 : (sizeof(F) == 4 ? 1 : 0);
    rec.lanes = h->lanes;
    rec.count = count;
    const int rows = spmv_rows(h->n, h->grid);
    rec.shm = h->halo > 0 ? (size_t)(rows + 2 * h->halo) * sizeof(F) : 0;
    rec.sp = SpmvSlot{h->n, h->halo, rows, h->grid, h->rp, h->ci, v, p, q, h->part_pq, h->st};
    rec.bj.P = P;
    rec.bj.Vv = Vv;
    rec.bj.st = h->st;
    rec.bj.it0 = it;
    rec.pu = PupdSlot{h->n, h->nb, pupdate_grid(h->n), it, p, z, h->part_rz, h->part_rr, h->st};
    h->defer->recs.push_back(rec);
    h->unflushed = true;
    h->holder = h->defer;
    batch_start = it;
    batch_count = count;
    sampled.clear();
    it += count;
}
}  // namespace

void sdsl_group_s::flush() {
    if (recs.empty()) return;
    // groups of one kernel instantiation, in first-appearance order; in a
    // group the slots go by decreasing iteration count, so that the slots
    // still iterating at offset k are a prefix of the table
    std::vector<std::vector<int>> parts;
    for (int i = 0; i < (int)recs.size(); ++i) {
        bool put = false;
        for (auto& g : parts)
            if (recs[g[0]].type == recs[i].type && recs[g[0]].lanes == recs[i].lanes) {
                g.push_back(i);
                put = true;
                break;
            }
        if (!put) parts.push_back({i});
    }
    for (auto& g : parts)
        std::stable_sort(g.begin(), g.end(), [&](int a, int b) { return recs[a].count > recs[b].count; });
    auto up = [](size_t x) { return (x + 63) / 64 * 64; };
    size_t bytes = 0;
    std::vector<size_t> base(parts.size());
    for (size_t gi = 0; gi < parts.size(); ++gi) {
        const size_t ns = parts[gi].size();
        base[gi] = bytes;
        bytes += up(3 * (ns + 1) * sizeof(int)) + up(ns * sizeof(SpmvSlot)) + up(ns * sizeof(BjSlot)) +
                 up(ns * sizeof(PupdSlot));
    }
    reserve(bytes);
    std::vector<SlotTable> tabs(parts.size());
    std::vector<std::vector<int>> pres(parts.size());
    for (size_t gi = 0; gi < parts.size(); ++gi) {
        const auto& g = parts[gi];
        const int ns = (int)g.size();
        char* hb = stage + base[gi];
        char* db = dev + base[gi];
        int* pre = (int*)hb;  // spmv_pre | bj_pre | pu_pre
        pre[0] = pre[ns + 1] = pre[2 * (ns + 1)] = 0;
        for (int i = 0; i < ns; ++i) {
            const IssueRec& r = recs[g[i]];
            pre[i + 1] = pre[i] + (r.sp.grid + 7) / 8 * 8;
            pre[ns + 1 + i + 1] = pre[ns + 1 + i] + r.bj.P.nblocks;
            pre[2 * (ns + 1) + i + 1] = pre[2 * (ns + 1) + i] + r.pu.grid;
        }
        size_t off = up(3 * (ns + 1) * sizeof(int));
        SpmvSlot* sp = (SpmvSlot*)(hb + off);
        const size_t o_sp = off;
        off += up(ns * sizeof(SpmvSlot));
        BjSlot* bj = (BjSlot*)(hb + off);
        const size_t o_bj = off;
        off += up(ns * sizeof(BjSlot));
        PupdSlot* pu = (PupdSlot*)(hb + off);
        const size_t o_pu = off;
        for (int i = 0; i < ns; ++i) {
            sp[i] = recs[g[i]].sp;
            bj[i] = recs[g[i]].bj;
            pu[i] = recs[g[i]].pu;
        }
        tabs[gi] = SlotTable{(const int*)db, (const SpmvSlot*)(db + o_sp), (const int*)db + (ns + 1),
                             (const BjSlot*)(db + o_bj), (const int*)db + 2 * (ns + 1), (const PupdSlot*)(db + o_pu)};
        pres[gi].assign(pre, pre + 3 * (ns + 1));
    }
    hip_check(hipMemcpyAsync(dev, stage, bytes, hipMemcpyHostToDevice, s), "copy");
    hip_check(hipEventRecord(copied, s), "event record");
    copy_pending = true;
    for (size_t gi = 0; gi < parts.size(); ++gi) {
        const auto& g = parts[gi];
        const int ns = (int)g.size();
        const IssueRec& r0 = recs[g[0]];
        size_t shm = 0;
        for (int i : g) shm = std::max(shm, recs[i].shm);
        const int* pre = pres[gi].data();
        auto issue_all = [&](hipStream_t st) {
            int live = ns;
            for (int k = 0; k < r0.count; ++k) {
                while (live > 0 && recs[g[live - 1]].count <= k) --live;
                const int wg[3] = {pre[live], pre[ns + 1 + live], pre[2 * (ns + 1) + live]};
                launch(r0.type, tabs[gi], live, k, r0.lanes, wg, shm, st);
            }
        };
        stats.flushes += 1;
        stats.slot_issues += ns;
        stats.launches += 3 * (int64_t)r0.count;
        if (!graphs) {
            issue_all(s);
            hip_check(hipGetLastError(), "kernel launch");
            continue;
        }
        // the graph of this shape: the kernels read the table, so only the
        // layout (types, counts, grids, window, table address) is its key
        std::vector<int64_t> key{r0.type, r0.lanes, ns, (int64_t)shm, (int64_t)(intptr_t)(dev + base[gi])};
        for (int i : g) key.push_back(recs[i].count);
        for (int q = 0; q < 3 * (ns + 1); ++q) key.push_back(pre[q]);
        Graph* hit = nullptr;
        for (auto& c : cache)
            if (c.key == key) hit = &c;
        if (!hit) {
            if (cache.size() >= 16) {
                auto lru = std::min_element(cache.begin(), cache.end(),
                                            [](const Graph& a, const Graph& b) { return a.used < b.used; });
                (void)hipGraphExecDestroy(lru->exec);
                cache.erase(lru);
            }
            hipGraph_t graph = nullptr;
            hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
            issue_all(cap);
            const hipError_t le = hipGetLastError();
            const hipError_t ce = hipStreamEndCapture(cap, &graph);
            hip_check(le, "kernel launch under capture");
            hip_check(ce, "end capture");
            hipGraphExec_t exec = nullptr;
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            hip_check(ie, "graph instantiate");
            cache.push_back(Graph{key, exec, 0});
            hit = &cache.back();
            stats.captures += 1;
        }
        hit->used = ++tick;
        hip_check(hipGraphLaunch(hit->exec, s), "graph launch");
        stats.graph_launches += 1;
    }
    for (auto& r : recs) {
        r.h->unflushed = false;
        r.h->holder = nullptr;
    }
    recs.clear();
}

void delete_group(sdsl_group_s* g) { delete g; }

// the one-handle group of a graphs = 1 handle: its stream and allocator
sdsl_group_s* make_own_group(sdsl_ctx* h) {
    std::unique_ptr<sdsl_group_s> g(new sdsl_group_s());
    g->s = h->s;
    g->graphs = true;
    g->al = h->al;
    hip_check(hipEventCreateWithFlags(&g->copied, hipEventDisableTiming), "event create");
    hip_check(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking), "stream create");
    return g.release();
}

namespace {

// sum of a device partial array into scal[idx], then copied to the host
double reduce_to_host(sdsl_ctx* h, const double* part, int m, int idx) {
    launch_sum_partials(part, m, h->scal + idx, h->s);
    h->check_launch();
    hip_check(hipMemcpyAsync(h->scal_h + idx, h->scal + idx, sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
    h->sync();
    return h->scal_h[idx];
}

// r = b - M x (compensated FP64); scal[0] = ||r||^2; returns ||r||
double true_residual(sdsl_ctx* h, const double* b, const double* x, double* r) {
    const CsrView A{h->n, h->rp, h->ci, h->halo};
    launch_residual(A, h->v, h->lr, b, x, r, h->part_res, h->lanes, h->grid, h->s);
    h->check_launch();
    return std::sqrt(reduce_to_host(h, h->part_res, h->grid, 0));
}

// FP64 operator y = M x (+ U diag(c) U^T x)
void apply_op64(sdsl_ctx* h, const double* x, double* y) {
    const CsrView A{h->n, h->rp, h->ci, h->halo};
    if (h->lr.k > 0) launch_lowrank_tdot<double>(h->lr, x, nullptr, LR_SCALED, h->s);
    launch_spmv<double, double>(A, h->v, h->lr, x, y, nullptr, nullptr, h->lanes, h->grid, h->s);
}

// FP64 preconditioner z = P^{-1} r (block Jacobi, with the border
// correction of the low-rank term when present)
void apply_prec64(sdsl_ctx* h, const double* r, double* z) {
    PcgVecs V{};
    V.r = const_cast<double*>(r);
    V.z = z;
    V.y = h->y;
    if (h->bbd) {
        // Sec. 2.4: w = L^{-1} r_I; g = r_G - F U_TT^{-1} w_T; x_G = S^{-1} g;
        // w_T -= L_TT^{-1} E_T x_G; z_I = U^{-1} w
        const int ni = h->n_int;
        launch_bj<double, double>(3, bj_dev(h, false), V, nullptr, 0, h->s);
        launch_bbd_mid(h->tdev, h->nb, h->bbd_max_nf, h->nbd, h->bbd_Sinv, h->bbd_fptr, h->bbd_fidx, h->bbd_gpart,
                       r + ni, h->bbd_g, h->y, z + ni, h->s);
        launch_bj<double, double>(4, bj_dev(h, false), V, nullptr, 0, h->s);
        return;
    }
    launch_bj<double, double>(0, bj_dev(h, false), V, nullptr, 0, h->s);
    if (h->bd.k > 0) {
        launch_lowrank_tdot<double>(h->lr, z, nullptr, LR_BORDER, h->s);
        launch_border_fix<double>(h->n, z, h->bd, h->s);
    }
}

__global__ void k_axpy1(int n, double* __restrict__ x, const double* __restrict__ d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = x[i] + d[i];
}

// ------------------------------------------------------------- refinement rule
// What the FP32 modes do at a refinement point (a tuned rule; the paper
// states no precision).  A point is weak when the true residual norm is above
// kRfWeak times that of the previous point; `slow` counts weak points in a
// row.  Mixed recurrence: converged -> done; a breakdown -> back to the last
// point's solution and FP64 solves of the residual equation; kRfHand weak
// points in a row -> FP64 solves of the residual equation from the current
// solution.  Classical refinement: an inner solve that broke down is
// discarded and FP64 solves of the residual equation follow; kRfSlow weak
// steps in a row -> FP64 solves of the residual equation.  Such a solve is a fresh FP64 PCG to
// kRfFbTol of the remaining tolerance; after it: converged -> done; another
// one when it converged and fewer than kRfMaxFb were run; otherwise fail.
enum RfAction { RF_DONE = 0, RF_CONTINUE = 1, RF_FALLBACK = 2, RF_REVERT = 3, RF_FAIL = 4 };
constexpr double kRfWeak = 0.5;
constexpr int kRfHand = 3;
constexpr int kRfSlow = 2;
constexpr int kRfMaxFb = 4;
constexpr double kRfFbTol = 0.5;
constexpr int kRfHistory = SDSL_RF_HISTORY;

int rf_decide(bool mixed, double nr, double prev, double tol_nb, bool breakdown, int& slow) {
    if (nr <= tol_nb) return RF_DONE;
    if (mixed) {
        slow = nr > kRfWeak * prev ? slow + 1 : 0;
        if (breakdown) return RF_REVERT;
        return slow >= kRfHand ? RF_FALLBACK : RF_CONTINUE;
    }
    if (breakdown) return RF_REVERT;
    slow = nr > kRfWeak * prev ? slow + 1 : 0;
    return slow >= kRfSlow ? RF_FALLBACK : RF_CONTINUE;
}

int fb_decide(double nr, double tol_nb, sdsl_status st64, int nsolves) {
    if (nr <= tol_nb) return RF_DONE;
    return (st64 == SDSL_OK && nsolves < kRfMaxFb) ? RF_FALLBACK : RF_FAIL;
}

// ------------------------------------------------------------- solve task
// Resumable solve: `step()` reads the state of the pending device work and
// issues the next stretch; sdsl_solve runs one task to the end,
// sdsl_solve_batch interleaves several tasks on their own streams.
struct SolveTask {
    sdsl_ctx* h = nullptr;
    const double* b = nullptr;
    double* user_x = nullptr;  // MC64: the caller's x = Dc y, written at the end
    double* xout = nullptr;
    double tol = 1e-8;
    double nb = 0.0;
    int total_its = 0, outer = 0, fallbacks = 0, restarts = 0;
    double relres = 1.0;
    sdsl_status status = SDSL_OK;
    bool finished = false;
    double t0 = 0.0;

    enum Phase { P64, PMIX, P32_RESTART, PGMRES, PBICG, PGCR } phase = P64;
    Pcg<double, double> pcg64{};
    Pcg<double, float> pcgmix{};
    Pcg<float, float> pcg32{};
    // FP64 PCG target (the solve itself, or an FP64 fallback of an FP32 mode)
    const double* rhs64 = nullptr;
    double* out64 = nullptr;
    double tol64 = 0.0, nrhs64 = 0.0;
    bool fallback = false;
    int fb_base_its = 0;
    // refinement bookkeeping
    double nr = 0.0, prev = 0.0;
    int slow = 0;
    int nsolves = 0;  // FP64 solves of the residual equation
    void record(int its, double res, int act, int flag) {
        sdsl_info& I = h->info;
        if (I.rf_count < kRfHistory) {
            I.rf_it[I.rf_count] = its;
            I.rf_nr[I.rf_count] = res;
            I.rf_act[I.rf_count] = act;
            I.rf_flag[I.rf_count] = flag;
        }
        I.rf_count++;
    }

    int max_iter() const { return h->o.max_iter; }

    void begin(sdsl_ctx* hh, const double* bb, double* xx, double tt) {
        h = hh; b = bb; xout = xx; tol = tt;
        if (h->mc64) {
            // Alg. 3: the Krylov method solves A' y = Q Dr b
            launch_mc64_rhs(h->n, h->m_rowof, h->m_rs, bb, h->m_b, h->s);
            h->check_launch();
            b = h->m_b;
            user_x = xx;
            xout = h->m_y;
        }
        t0 = now_ms();
        for (int p = 0; p < 2; ++p) {
            h->info.spmv_ms[p] = h->info.bj_ms[p] = 0.0;
            h->info.spmv_launches[p] = h->info.bj_launches[p] = 0;
        }
        h->info.rf_count = 0;
        launch_sqnorm_partials(h->n, b, h->part_b, h->grid, h->s);
        h->check_launch();
        nb = std::sqrt(reduce_to_host(h, h->part_b, h->grid, 1));  // scal[1] = ||b||^2
        h->info.rf_nb = nb;
        launch_fill<double>(h->n, xout, 0.0, h->s);
        if (nb == 0.0) { finish(SDSL_OK, 0.0); return; }
        pcg64 = Pcg<double, double>{h, h->x, h->r, h->z, h->p, h->q, h->y, h->v};
        pcg64.init();
        pcgmix = Pcg<double, float>{h, xout, h->r, h->z, h->p, h->q, h->y32, h->v32};
        pcgmix.init();
        pcg32 = Pcg<float, float>{h, h->x32, h->r32, h->z32, h->p32, h->q32, h->y32, h->v32};
        pcg32.init();
        if (h->o.krylov == SDSL_GMRES) {
            gm_begin();
        } else if (h->o.krylov == SDSL_GCR) {
            gcr_begin();
        } else if (h->o.krylov == SDSL_BICGSTAB) {
            bi_begin();
        } else if (h->o.precision == SDSL_FP64) {
            start64(b, xout, tol, nb);
        } else if (h->o.precision == SDSL_FP32_IR) {
            // FP64 recurrence over the FP32 operator and factors; the true
            // FP64 residual replaces the recurrence one at refinement points
            phase = PMIX;
            nr = prev = nb;
            launch_copy<double>(h->n, b, h->r, h->s);
            launch_fill<double>(h->n, h->xref, 0.0, h->s);
            launch_init_state(h->st, h->part_b, h->grid, tol, h->o.refine_delta, h->s);
            launch_refine_state(h->st, h->part_b, h->grid, 0, h->o.refine_every, h->s);
            pcgmix.start(0);
            pcgmix.issue(std::min(h->o.check_every, max_iter()));
        } else {
            phase = P32_RESTART;
            nr = true_residual(h, b, xout, h->r);
            if (nr <= tol * nb) { finish(SDSL_OK, nr / nb); return; }
            restart_inner();
        }
    }
    void finish(sdsl_status s, double rr) {
        status = s;
        relres = rr;
        finished = true;
        if (user_x) {
            launch_mc64_sol(h->n, h->m_cs, xout, user_x, h->s);  // x = Dc y
            h->check_launch();
            h->sync();
        }
        h->info.solve_ms = now_ms() - t0;
        h->info.relres = rr;
        h->info.inner_iters = total_its;
        h->info.outer_iters = outer;
        h->info.fp64_fallbacks = fallbacks;
        h->info.restarts = restarts;
    }
    // FP64 PCG on M out = rhs, x0 = 0, to ||rhs - M out|| <= t * nrhs
    void start64(const double* rhs, double* out, double t, double nrhs) {
        phase = P64;
        rhs64 = rhs;
        out64 = out;
        tol64 = t;
        nrhs64 = nrhs;
        pcg64.set_x(out);
        launch_fill<double>(h->n, out, 0.0, h->s);
        launch_copy<double>(h->n, rhs, h->r, h->s);
        launch_sqnorm_partials(h->n, rhs, h->part_res, h->grid, h->s);
        launch_init_state(h->st, h->part_res, h->grid, t, 0.0, h->s);
        pcg64.start(0);
        pcg64.issue(std::min(h->o.check_every, std::max(1, max_iter() - total_its)));
    }
    // FP64 fallback of the FP32 modes: solve M d = r (the current residual)
    void start_fallback() {
        fallback = true;
        fallbacks++;
        nsolves++;
        fb_base_its = total_its;
        launch_copy<double>(h->n, h->r, h->rf, h->s);
        // part of the needed reduction, so that the rounding of x += d keeps
        // the true residual below the tolerance
        start64(h->rf, h->d, kRfFbTol * tol * nb / nr, nr);
    }
    void restart_inner() {
        // classical refinement: inner FP32 PCG on M d = r / ||r|| to inner_tol
        if (outer >= h->o.max_outer || total_its >= max_iter()) { finish(SDSL_E_NOT_CONVERGED, nr / nb); return; }
        launch_ir_scale_cast(h->n, h->r, h->scal + 0, h->r32, h->s);
        launch_fill<float>(h->n, h->x32, 0.0f, h->s);
        launch_sqnorm_f32_partials(h->n, h->r32, h->part_res, h->grid, h->s);
        launch_init_state(h->st, h->part_res, h->grid, h->o.inner_tol, 0.0, h->s);
        pcg32.start(0);
        pcg32.issue(inner_batch());
    }
    // iterations of the next batch of a classical-refinement inner solve: it
    // stops at inner_tol, after refine_every iterations or at max_iter
    int inner_batch() const {
        return std::max(0, std::min({h->o.check_every, max_iter() - total_its - pcg32.it,
                                     h->o.refine_every - pcg32.it}));
    }
    void after_fallback(sdsl_status st64) {
        const int g = std::min(4096, (h->n + 255) / 256);
        k_axpy1<<<std::max(g, 1), 256, 0, h->s>>>(h->n, xout, h->d);  // x += d
        h->check_launch();
        nr = true_residual(h, b, xout, h->r);
        fallback = false;
        const int act = (total_its >= max_iter() && nr > tol * nb) ? RF_FAIL : fb_decide(nr, tol * nb, st64, nsolves);
        record(total_its, nr, act, 2);
        if (act == RF_DONE) { finish(SDSL_OK, nr / nb); return; }
        if (act == RF_FALLBACK) { start_fallback(); return; }
        finish(st64 == SDSL_E_BREAKDOWN ? SDSL_E_BREAKDOWN : SDSL_E_NOT_CONVERGED, nr / nb);
    }

    // ---- GMRES(m), right preconditioned, FP64 (Sec. 2.2): Arnoldi with
    // classical Gram-Schmidt applied twice, Givens rotations on the host,
    // x += Z y at the end of a cycle, restart from the true residual
    int gm_m = 0, gm_j = 0;
    std::vector<double> gH, gcs, gsn, gg;
    void gm_begin() {
        phase = PGMRES;
        gm_alloc();
        gH.assign((size_t)(gm_m + 1) * gm_m, 0.0);
        gcs.assign(gm_m, 0.0);
        gsn.assign(gm_m, 0.0);
        gg.assign(gm_m + 1, 0.0);
        gm_cycle();
    }
    // the restart length and the basis storage: V (m + 1 columns), Z (m)
    void gm_alloc() {
        gm_m = std::max(1, std::min(h->o.restart, kMaxBasisHost - 1));
        const int n = h->n;
        if (h->gm_cap < gm_m) {
            h->gV = h->alloc<double>((size_t)(gm_m + 1) * n);
            h->gZ = h->alloc<double>((size_t)gm_m * n);
            if (!h->gpart) {
                h->gpart = h->alloc<double>((size_t)512 * kMaxBasisHost);
                h->gnrm = h->alloc<double>(512);
                h->ghcol = h->alloc<double>(kMaxBasisHost);
                h->gh2 = h->alloc<double>(kMaxBasisHost);
                h->gy = h->alloc<double>(kMaxBasisHost);
                hip_check(hipHostMalloc((void**)&h->gh_h, (kMaxBasisHost + 2) * sizeof(double), hipHostMallocDefault),
                          "pinned alloc");
            }
            h->gm_cap = gm_m;
        }
    }
    void gm_cycle() {
        // r = b - M x (compensated), scal[0] = ||r||^2
        nr = true_residual(h, b, xout, h->r);
        if (nr <= tol * nb) { finish(SDSL_OK, nr / nb); return; }
        if (total_its >= max_iter()) { finish(SDSL_E_NOT_CONVERGED, nr / nb); return; }
        if (outer > 0) restarts++;
        outer++;
        launch_scale_inv_norm(h->n, h->scal + 0, h->r, h->gV, h->s);
        std::fill(gg.begin(), gg.end(), 0.0);
        gg[0] = nr;
        gm_j = 0;
    }
    void gm_step() {
        const int n = h->n, j = gm_j;
        double* vj = h->gV + (size_t)j * n;
        double* zj = h->gZ + (size_t)j * n;
        double* w = h->gV + (size_t)(j + 1) * n;
        apply_prec64(h, vj, zj);
        apply_op64(h, zj, w);
        launch_multidot(n, j + 1, h->gV, n, w, h->gpart, h->ghcol, nullptr, h->s);
        launch_multiaxpy(n, j + 1, h->gV, n, h->ghcol, -1.0, w, nullptr, h->s);
        launch_multidot(n, j + 1, h->gV, n, w, h->gpart, h->gh2, h->ghcol, h->s);
        launch_multiaxpy(n, j + 1, h->gV, n, h->gh2, -1.0, w, h->gnrm, h->s);
        launch_sum_partials(h->gnrm, 512, h->scal + 2, h->s);
        h->check_launch();
        hip_check(hipMemcpyAsync(h->gh_h, h->ghcol, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
        hip_check(hipMemcpyAsync(h->gh_h + kMaxBasisHost, h->scal + 2, sizeof(double), hipMemcpyDeviceToHost, h->s),
                  "copy");
        h->sync();
        double* col = &gH[(size_t)j * (gm_m + 1)];
        for (int i = 0; i <= j; ++i) col[i] = h->gh_h[i];
        const double hn = std::sqrt(h->gh_h[kMaxBasisHost]);
        col[j + 1] = hn;
        double cnorm = 0.0;
        for (int i = 0; i <= j + 1; ++i) cnorm = std::max(cnorm, std::fabs(col[i]));
        for (int i = 0; i < j; ++i) {
            const double a = col[i], c = col[i + 1];
            col[i] = gcs[i] * a + gsn[i] * c;
            col[i + 1] = -gsn[i] * a + gcs[i] * c;
        }
        const double t = col[j], u = col[j + 1];
        const double rr = std::hypot(t, u);
        gcs[j] = rr > 0.0 ? t / rr : 1.0;
        gsn[j] = rr > 0.0 ? u / rr : 0.0;
        col[j] = rr;
        col[j + 1] = 0.0;
        gg[j + 1] = -gsn[j] * gg[j];
        gg[j] = gcs[j] * gg[j];
        total_its++;
        gm_j = j + 1;
        const bool happy = !(hn > 1e-14 * cnorm);
        if (!happy) launch_scale_inv_norm(n, h->scal + 2, w, w, h->s);
        if (std::fabs(gg[j + 1]) <= tol * nb || happy || gm_j == gm_m || total_its >= max_iter()) gm_update();
    }
    void gm_update() {
        // y = R^{-1} g by back substitution; x += Z y
        const int k = gm_j;
        std::vector<double> yv(k, 0.0);
        for (int i = k - 1; i >= 0; --i) {
            double s = gg[i];
            for (int c = i + 1; c < k; ++c) s -= gH[(size_t)c * (gm_m + 1) + i] * yv[c];
            const double d = gH[(size_t)i * (gm_m + 1) + i];
            yv[i] = d != 0.0 ? s / d : 0.0;
        }
        for (int i = 0; i < k; ++i) h->gh_h[i] = yv[i];
        hip_check(hipMemcpyAsync(h->gy, h->gh_h, k * sizeof(double), hipMemcpyHostToDevice, h->s), "copy");
        launch_multiaxpy(h->n, k, h->gZ, h->n, h->gy, 1.0, xout, nullptr, h->s);
        h->check_launch();
        gm_cycle();
    }

    // ---- GCR(m), right preconditioned, FP64 (Sec. 2.2; the paper's solver
    // with BBD, Sec. 4.2-4.3): directions P = Z columns, Q = M P = V
    // columns, Q orthonormal within a cycle (classical Gram-Schmidt applied
    // twice, the same coefficients update P).  The host reads ||q|| and
    // ||r|| once per step; every cycle starts from the true residual.
    int gcr_j = 0;
    void gcr_begin() {
        phase = PGCR;
        gm_alloc();
        gcr_cycle();
    }
    void gcr_cycle() {
        nr = true_residual(h, b, xout, h->r);
        if (nr <= tol * nb) { finish(SDSL_OK, nr / nb); return; }
        if (total_its >= max_iter()) { finish(SDSL_E_NOT_CONVERGED, nr / nb); return; }
        if (outer > 0) restarts++;
        outer++;
        gcr_j = 0;
    }
    void gcr_step() {
        const int n = h->n, j = gcr_j;
        double* pj = h->gZ + (size_t)j * n;
        double* qj = h->gV + (size_t)j * n;
        apply_prec64(h, h->r, pj);
        apply_op64(h, pj, qj);
        // (q, Q_i) for i < j and (q, q) in ghcol[j]: Q_j is column j of V
        launch_multidot(n, j + 1, h->gV, n, qj, h->gpart, h->ghcol, nullptr, h->s);
        const double* nu2 = h->ghcol + j;
        if (j > 0) {
            launch_multiaxpy(n, j, h->gV, n, h->ghcol, -1.0, qj, nullptr, h->s);
            launch_multiaxpy(n, j, h->gZ, n, h->ghcol, -1.0, pj, nullptr, h->s);
            launch_multidot(n, j, h->gV, n, qj, h->gpart, h->gh2, nullptr, h->s);
            launch_multiaxpy(n, j, h->gV, n, h->gh2, -1.0, qj, h->gnrm, h->s);
            launch_multiaxpy(n, j, h->gZ, n, h->gh2, -1.0, pj, nullptr, h->s);
            launch_sum_partials(h->gnrm, 512, h->scal + 2, h->s);
            nu2 = h->scal + 2;
        }
        const int g = bicg_grid(n);
        double* part_rq = h->gpart;
        double* part_rr = h->gpart + 4096;
        launch_dot2(n, h->r, qj, nullptr, nullptr, part_rq, nullptr, nullptr, h->s);
        launch_gcr_xr(n, xout, h->r, pj, qj, nu2, h->ghcol + j, part_rq, part_rr, h->s);
        launch_sum_partials(part_rr, g, h->scal + 3, h->s);
        h->check_launch();
        hip_check(hipMemcpyAsync(h->gh_h, nu2, sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
        hip_check(hipMemcpyAsync(h->gh_h + 1, h->ghcol + j, sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
        hip_check(hipMemcpyAsync(h->gh_h + 2, h->scal + 3, sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
        h->sync();
        const double v2 = h->gh_h[0], v02 = h->gh_h[1], rn = std::sqrt(h->gh_h[2]);
        if (!(v2 > 1e-28 * v02) || !std::isfinite(v2)) {
            // the new direction adds nothing: x and r were left unchanged
            nr = true_residual(h, b, xout, h->r);
            finish(nr <= tol * nb ? SDSL_OK : SDSL_E_BREAKDOWN, nr / nb);
            return;
        }
        total_its++;
        gcr_j = j + 1;
        if (rn <= tol * nb || gcr_j == gm_m || total_its >= max_iter()) gcr_cycle();
    }

    // ---- BiCGSTAB, right preconditioned, FP64 (Sec. 2.2, Sec. 4.3): the
    // vector steps keep every scalar on the device (k_bicg_*); the host
    // issues check_every iterations between polls.  Vectors: r^ in rf, p,
    // v in q, p^ = P^{-1} p in z, s in d, s^ = P^{-1} s in xref, t in x.
    int bi_it = 0;
    bool bi_first = true;
    double* bp_(int k) { return h->bi_part + (size_t)k * bicg_grid(h->n); }
    void bi_prec(const double* in, double* out) {
        PcgVecs V{};
        V.r = const_cast<double*>(in);
        V.z = out;
        V.y = h->y;
        launch_bj<double, double>(0, bj_dev(h, false), V, h->st, 0, h->s);
        if (h->bd.k > 0) {
            launch_lowrank_tdot<double>(h->lr, out, h->st, LR_BORDER, h->s);
            launch_border_fix<double>(h->n, out, h->bd, h->s);
        }
    }
    void bi_op(const double* in, double* out) {
        const CsrView A{h->n, h->rp, h->ci, h->halo};
        if (h->lr.k > 0) launch_lowrank_tdot<double>(h->lr, in, h->st, LR_SCALED, h->s);
        launch_spmv<double, double>(A, h->v, h->lr, in, out, nullptr, h->st, h->lanes, h->grid, h->s);
    }
    // a cycle from the residual in r: r^ = r, partials of (r^, r), ||r||^2
    void bi_cycle_start() {
        launch_copy<double>(h->n, h->r, h->rf, h->s);
        launch_dot2(h->n, h->rf, h->r, h->r, h->r, bp_(0), bp_(1), nullptr, h->s);
        bi_first = true;
    }
    void bi_begin() {
        phase = PBICG;
        launch_copy<double>(h->n, b, h->r, h->s);
        launch_init_state(h->st, h->part_b, h->grid, tol, 0.0, h->s);
        bi_cycle_start();
        bi_issue(std::min(h->o.check_every, max_iter()));
    }
    void bi_issue(int count) {
        const int n = h->n;
        for (int k = 0; k < count; ++k, ++bi_it) {
            launch_bicg_p(n, h->r, h->p, h->q, bp_(0), bp_(1), h->st, bi_it, bi_first, h->s);
            bi_first = false;
            bi_prec(h->p, h->z);
            bi_op(h->z, h->q);
            launch_dot2(n, h->rf, h->q, nullptr, nullptr, bp_(2), nullptr, h->st, h->s);
            launch_bicg_s(n, h->r, h->q, h->d, bp_(2), bp_(3), h->st, bi_it, h->s);
            bi_prec(h->d, h->xref);
            bi_op(h->xref, h->x);
            launch_dot2(n, h->x, h->d, h->x, h->x, bp_(4), bp_(5), h->st, h->s);
            launch_bicg_x(n, xout, h->z, h->xref, h->d, h->x, h->r, h->rf, bp_(3), bp_(4), bp_(5), bp_(0), bp_(1),
                          h->st, bi_it, h->s);
        }
        h->check_launch();
    }
    void bi_step() {
        hip_check(hipMemcpyAsync(h->st_h, h->st, sizeof(KrylovState), hipMemcpyDeviceToHost, h->s), "copy");
        h->sync();
        const KrylovState s = *h->st_h;
        if (!s.done) {
            if (bi_it >= max_iter()) {
                total_its = bi_it;
                nr = true_residual(h, b, xout, h->r);
                finish(SDSL_E_NOT_CONVERGED, nr / nb);
                return;
            }
            bi_issue(std::min(h->o.check_every, max_iter() - bi_it));
            return;
        }
        total_its = s.iters;
        nr = true_residual(h, b, xout, h->r);
        if (s.breakdown) { finish(SDSL_E_BREAKDOWN, nr / nb); return; }
        if (nr <= tol * nb) { finish(SDSL_OK, nr / nb); return; }
        if (total_its >= max_iter()) { finish(SDSL_E_NOT_CONVERGED, nr / nb); return; }
        // the recurrence met the tolerance but the true residual (now in r)
        // did not: a new cycle from it
        restarts++;
        bi_it = total_its;
        launch_init_state(h->st, h->part_b, h->grid, tol, 0.0, h->s);
        bi_cycle_start();
        bi_issue(std::min(h->o.check_every, max_iter() - bi_it));
    }

    void step() {
        if (finished) return;
        if (phase == PGMRES) { gm_step(); return; }
        if (phase == PBICG) { bi_step(); return; }
        if (phase == PGCR) { gcr_step(); return; }
        if (phase == P64) { step64(); return; }
        if (phase == PMIX) { step_mixed(); return; }
        // classical refinement: wait for the inner solve to stop
        const KrylovState& s = pcg32.poll();
        if (!s.done && inner_batch() > 0) {
            pcg32.issue(inner_batch());
            return;
        }
        const int inner = s.done ? s.iters : pcg32.it;
        total_its += inner;
        const bool bd = s.done && s.breakdown;
        outer++;
        prev = nr;
        if (!bd) {
            launch_ir_update(h->n, xout, h->scal + 0, h->x32, h->s);   // x += ||r|| d
            h->check_launch();
            nr = true_residual(h, b, xout, h->r);
        }
        const int act = rf_decide(false, nr, prev, tol * nb, bd, slow);
        record(total_its, nr, act, bd ? 1 : 0);
        if (act == RF_DONE) { finish(SDSL_OK, nr / nb); return; }
        if (act == RF_FALLBACK || act == RF_REVERT) { start_fallback(); return; }
        restart_inner();
    }
    void step_mixed() {
        const KrylovState& s = pcgmix.poll();
        const int it_now = pcgmix.it;
        if (!s.done) {
            if (it_now < max_iter()) {
                pcgmix.issue(std::min(h->o.check_every, max_iter() - it_now));
                return;
            }
            // the iteration limit without a refinement point
            total_its = it_now;
            nr = true_residual(h, b, xout, h->r);
            finish(SDSL_E_NOT_CONVERGED, nr / nb);
            return;
        }
        // refinement point: the true residual of the FP64 solution
        const int its = s.iters;
        total_its = its;
        outer++;
        prev = nr;
        nr = true_residual(h, b, xout, h->r);
        const bool bd = s.breakdown != 0;
        const int act = rf_decide(true, nr, prev, tol * nb, bd, slow);
        record(its, nr, act, bd ? 1 : 0);
        if (act == RF_DONE) { finish(SDSL_OK, nr / nb); return; }
        if (act == RF_REVERT) {
            // (p, Mp) <= 0 or a non-finite step: the FP32 operator or factors
            // are not positive definite for this system, so the search
            // direction is not continued: back to the solution of the last
            // refinement point (the steps since may already have gone
            // astray), then FP64 PCG solves the residual equation
            launch_copy<double>(h->n, h->xref, xout, h->s);
            nr = true_residual(h, b, xout, h->r);
            start_fallback();
            return;
        }
        if (act == RF_FALLBACK) { start_fallback(); return; }
        if (its >= max_iter()) { finish(SDSL_E_NOT_CONVERGED, nr / nb); return; }
        // the true residual (now in r) replaces the recurrence one; the
        // recurrence continues with its search direction
        launch_copy<double>(h->n, xout, h->xref, h->s);
        launch_refine_state(h->st, h->part_res, h->grid, its, h->o.refine_every, h->s);
        pcgmix.reapply(its - 1);
        pcgmix.issue(std::min(h->o.check_every, max_iter() - its));
    }
    void step64() {
        const KrylovState& s = pcg64.poll();
        const int used = pcg64.it;
        const int base = fallback ? fb_base_its : 0;
        if (!s.done) {
            if (base + used >= max_iter()) {
                total_its = base + used;
                end64(SDSL_E_NOT_CONVERGED);
                return;
            }
            pcg64.issue(std::min(h->o.check_every, max_iter() - base - used));
            return;
        }
        total_its = base + s.iters;
        if (s.breakdown) { end64(SDSL_E_BREAKDOWN); return; }
        // converged on the recurrence: check the true residual
        const double rr = true_residual(h, rhs64, out64, h->r);
        if (rr <= tol64 * nrhs64) { end64(SDSL_OK, rr); return; }
        if (total_its >= max_iter()) { end64(SDSL_E_NOT_CONVERGED, rr); return; }
        // restart from the true residual (now in r); the solution keeps accumulating
        restarts++;
        launch_sqnorm_partials(h->n, rhs64, h->part_res, h->grid, h->s);
        launch_init_state(h->st, h->part_res, h->grid, tol64, 0.0, h->s);
        pcg64.start(s.iters);
        pcg64.issue(std::min(h->o.check_every, max_iter() - base - s.iters));
    }
    void end64(sdsl_status st, double rr = -1.0) {
        if (fallback) { after_fallback(st); return; }
        if (rr < 0) rr = true_residual(h, rhs64, out64, h->r);
        finish(st, rr / nb);
    }
};

void delete_task(SolveTask* t) { delete t; }

sdsl_status guard(sdsl_ctx* h, const std::function<void()>& fn) {
    try {
        fn();
        if (h) h->err.clear();
        return SDSL_OK;
    } catch (const Error& e) {
        if (h) h->err = e.msg;
        g_thread_err = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        if (h) h->err = "host allocation failed";
        g_thread_err = "host allocation failed";
        return SDSL_E_NOMEM;
    } catch (...) {
        if (h) h->err = "unexpected internal error";
        g_thread_err = "unexpected internal error";
        return SDSL_E_DEVICE;
    }
}

// one running solve per handle: calls that use the handle's vectors or
// factors are refused while an asynchronous solve is unfinished
void check_idle(sdsl_ctx* h) {
    if (h->task && !h->task->finished) fail(SDSL_E_STATE, "an asynchronous solve is running on this handle");
}

void check_options(const sdsl_options* o) {
    if (o->method != SDSL_BJ && o->method != SDSL_BBD) fail(SDSL_E_INVALID, "unknown method");
    if (o->method == SDSL_BBD && ((o->krylov != SDSL_GMRES && o->krylov != SDSL_GCR) || o->precision != SDSL_FP64))
        fail(SDSL_E_INVALID, "the BBD preconditioner runs with GMRES or GCR in FP64");
    if (o->filter < SDSL_FILTER_NONE || o->filter > SDSL_FILTER_GEOMEAN) fail(SDSL_E_INVALID, "unknown filter");
    if (!(o->tau >= 0.0)) fail(SDSL_E_INVALID, "tau must be >= 0");
    if (!(o->delta >= 0.0) || !std::isfinite(o->delta)) fail(SDSL_E_INVALID, "delta must be finite and >= 0");
    if (o->pivot < SDSL_PIVOT_FAIL || o->pivot > SDSL_PIVOT_SHIFT) fail(SDSL_E_INVALID, "unknown pivot policy");
    if (o->pivot == SDSL_PIVOT_SHIFT && !(o->shift0 > 0.0 && std::isfinite(o->shift0)))
        fail(SDSL_E_INVALID, "shift0 must be positive");
    if (o->krylov != SDSL_PCG && o->krylov != SDSL_GMRES && o->krylov != SDSL_BICGSTAB && o->krylov != SDSL_GCR)
        fail(SDSL_E_INVALID, "unknown Krylov method");
    if (o->krylov == SDSL_GCR && o->precision != SDSL_FP64)
        fail(SDSL_E_INVALID, "GCR runs in FP64 (precision must be SDSL_FP64)");
    if (o->krylov == SDSL_GCR && (o->restart < 1 || o->restart >= kMaxBasisHost))
        fail(SDSL_E_INVALID, "GCR restart must be in [1, 63]");
    if (o->krylov == SDSL_BICGSTAB && (o->method != SDSL_BJ || o->precision != SDSL_FP64))
        fail(SDSL_E_INVALID, "BiCGSTAB runs with the block-Jacobi preconditioner in FP64");
    if (o->krylov == SDSL_GMRES && o->precision != SDSL_FP64)
        fail(SDSL_E_INVALID, "GMRES runs in FP64 (precision must be SDSL_FP64)");
    if (o->krylov == SDSL_GMRES && (o->restart < 1 || o->restart >= kMaxBasisHost))
        fail(SDSL_E_INVALID, "GMRES restart must be in [1, 63]");
    if (o->max_iter < 1 || o->check_every < 1) fail(SDSL_E_INVALID, "max_iter and check_every must be >= 1");
    if (o->mc64 != 0 && o->mc64 != 1) fail(SDSL_E_INVALID, "mc64 must be 0 or 1");
    if (o->mc64 && o->method != SDSL_BJ) fail(SDSL_E_INVALID, "MC64 applies to the block-Jacobi method");
    if (o->factor != SDSL_FACT_ILU0 && o->factor != SDSL_FACT_COMPLETE) fail(SDSL_E_INVALID, "unknown factorisation");
    if (o->graphs != 0 && o->graphs != 1) fail(SDSL_E_INVALID, "graphs must be 0 or 1");
    if (o->precision < SDSL_FP64 || o->precision > SDSL_FP32_IR_RESTART) fail(SDSL_E_INVALID, "unknown precision");
    if (o->precision == SDSL_FP32_IR_RESTART && (!(o->inner_tol > 0.0 && o->inner_tol < 1.0) || o->max_outer < 1))
        fail(SDSL_E_INVALID, "inner_tol must be in (0,1) and max_outer >= 1");
    if (o->precision == SDSL_FP32_IR && (!(o->refine_delta > 0.0 && o->refine_delta < 1.0) || o->refine_every < 1))
        fail(SDSL_E_INVALID, "refine_delta must be in (0,1) and refine_every >= 1");
}

void check_partition(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o) {
    if (!A || !p || !o) fail(SDSL_E_INVALID, "null argument");
    if (A->n <= 0) fail(SDSL_E_INVALID, "n must be positive");
    if (A->nnz < A->n || A->nnz > 0x7fffffffLL) fail(SDSL_E_INVALID, "nnz out of range (diagonal required, < 2^31)");
    if (!A->row_ptr || !A->col || !A->val) fail(SDSL_E_INVALID, "null CSR array");
    if (A->mem != SDSL_MEM_DEVICE && A->mem != SDSL_MEM_HOST) fail(SDSL_E_INVALID, "unknown memory kind");
    if (p->nblocks < 1 || !p->block_ptr) fail(SDSL_E_INVALID, "need at least one block");
    if (p->n_border < 0 || p->n_border >= A->n) fail(SDSL_E_INVALID, "bad n_border");
    if (o->method == SDSL_BJ && p->n_border != 0) fail(SDSL_E_INVALID, "block Jacobi takes no border");
    const int n_int = A->n - p->n_border;
    if (p->block_ptr[0] != 0 || p->block_ptr[p->nblocks] != n_int)
        fail(SDSL_E_INVALID, "block_ptr must start at 0 and end at n - n_border");
    for (int b = 0; b < p->nblocks; ++b)
        if (p->block_ptr[b + 1] <= p->block_ptr[b]) fail(SDSL_E_INVALID, "block_ptr must increase strictly");
}

}  // namespace

// -------------------------------------------- allocation-free residual
// sdsl_residual_noalloc keeps its reduction partials in this file-scope
// array instead of the handle's buffers: kNoAllocDoubles FP64 values
// (128 KiB) on every device the library runs on, held until the process
// ends.  Host code never passes `scratch` itself to a kernel (in host code
// the name is only a stand-in): the device address is taken once per device
// with hipGetSymbolAddress and kept in g_scratch.
constexpr size_t kNoAllocDoubles = 16384;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_scratch_mu;
double* g_scratch[kNoAllocDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
double* scratch_here() {
    int dev = -1;
    hip_check(hipGetDevice(&dev), "get device");
    if (dev < 0 || dev >= kNoAllocDevices) fail(SDSL_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "address of the residual scratch");
        if (!ptr) fail(SDSL_E_DEVICE, "no device address for the residual scratch");
        g_scratch[dev] = (double*)ptr;
    }
    return g_scratch[dev];
}
}  // namespace

// ===================================================================== C ABI
extern "C" {

void sdsl_default_options(sdsl_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = SDSL_BJ;
    o->filter = SDSL_FILTER_NONE;
    o->tau = 0.0;
    o->diag_flags = 0;
    o->delta = 0.0;
    o->pivot = SDSL_PIVOT_SHIFT;
    o->shift0 = 1e-2;
    o->spd = 1;
    o->krylov = SDSL_PCG;
    o->restart = 30;
    o->max_iter = 100000;
    o->precision = SDSL_FP64;
    o->inner_tol = 1e-4;
    o->max_outer = 30;
    o->check_every = 16;
    o->kernel_timing = 0;
    o->border = 1;
    o->refine_delta = 0.1;
    o->refine_every = 500;
}

size_t sdsl_footprint_bytes(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o,
                            const sdsl_lowrank* lr) {
    if (!A || !p || !o || A->n <= 0 || A->nnz < 0) return 0;
    const size_t n = (size_t)A->n, nnz = (size_t)A->nnz, nb = (size_t)std::max(p->nblocks, 1);
    size_t b = 0;
    b += (n + 1) * (8 + 4) + nnz * (4 + 8 + 4) + n * 8;            // operator + FP32 copy + diag
    if (o->mc64) b += nnz * (4 + 8) + n * (4 + 4 * 8);              // MC64 maps, scalings, b', y
    b += (n + 1) * 4 + nnz * (4 + 8 + 8) + n * (4 + 4 + 4 + 8);     // filtered pattern, values, factors
    // split factors (L and U each sized for every entry) + FP32 copies, the
    // U diagonal, chunk tables, levels
    b += (size_t)2 * nnz * (4 + 8 + 4) + 2 * (n + 1) * 4 + n * (8 + 4 + 2 * (8 + 4 + 4)) + 2 * nb * 12;
    b += (size_t)2 * n * kBjEllWidth * (4 + 8 + 4);                 // interleaved newest entries (L, U)
    b += (size_t)2 * ((n + 1) * 4 + nnz * (4 + 8 + 4));             // older entries (L, U)
    b += (size_t)2 * n * (8 + 4);                                   // level-order placement
    b += n * (9 * 8 + 6 * 4);                                       // Krylov vectors
    b += (size_t)6 * 4096 * 8;                                      // BiCGSTAB partials
    b += (nb + 1) * 4 + nb * (8 + 4) + 2048 * 8 * 4 + nb * 8 * 3;
    if (lr && lr->k > 0)  // U twice (CSR, CSC), W = P^{-1} U, K and its inverse, reduction partials
        b += (size_t)lr->U.nnz * 2 * (4 + 8) + (n + 1) * 4 + (size_t)lr->k * n * 8 + (size_t)lr->k * lr->k * 16 +
             64 * 1024;
    b += (n + 1023) / 1024 * 4 + 4096;
    if (o->krylov == SDSL_GMRES || o->krylov == SDSL_GCR) {
        // GMRES: basis V (m + 1 columns), Z = P^{-1} V (m columns); GCR: Q and
        // P in the same storage; reduction partials
        const size_t m = (size_t)std::max(1, std::min(o->restart, kMaxBasisHost - 1));
        b += (2 * m + 1) * n * 8 + ((size_t)512 * kMaxBasisHost + 512 + 3 * kMaxBasisHost) * 8;
    }
    if (o->method == SDSL_BBD) {
        // the tail factors depend on the pattern, which must be readable here
        const int nbd = p->n_border, ni = A->n - nbd;
        if (A->mem != SDSL_MEM_HOST || !A->row_ptr || !A->col || !p->block_ptr || nbd <= 0 || ni <= 0 ||
            p->nblocks <= 0 || A->nnz > INT32_MAX)
            return 0;
        const int64_t* rp = A->row_ptr;
        if (rp[0] != 0 || rp[A->n] != A->nnz) return 0;
        for (int i = 0; i < A->n; ++i)
            if (rp[i + 1] < rp[i]) return 0;
        for (int64_t q = 0; q < A->nnz; ++q)
            if (A->col[q] < 0 || A->col[q] >= A->n) return 0;
        const std::vector<int> bp(p->block_ptr, p->block_ptr + p->nblocks + 1);
        if (bp[0] != 0 || bp[p->nblocks] != ni) return 0;
        for (int q = 0; q < p->nblocks; ++q)
            if (bp[q + 1] < bp[q]) return 0;
        BbdPattern P;
        if (bbd_pattern(A->n, ni, bp, rp, A->col, P) >= 0) return 0;
        size_t hg = 0, sne = 0, snf = 0;
        for (int q = 0; q < p->nblocks; ++q) {
            const size_t t = (size_t)(bp[q + 1] - P.tail[q]);
            hg += t * (P.ecols[q].size() + P.frows[q].size());
            sne += P.ecols[q].size();
            snf += P.frows[q].size();
        }
        size_t ne = 0, nf = 0, nc = 0;  // entries of E, F and the border block C
        for (int i = 0; i < A->n; ++i)
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
                const bool bc = A->col[q] >= ni;
                if (i < ni) ne += bc;
                else if (bc) ++nc;
                else ++nf;
            }
        b += hg * 8;                                       // tail factors H and Gt
        b += (ne + nf + nc) * 2 * 8;                       // entry positions and targets
        b += (size_t)2 * nbd * nbd * 8 + (size_t)nbd * (2 * 4 + 8 + 4) + 4;  // S, S^{-1}, pivots, order, g, fptr
        b += (sne + 2 * snf) * 4 + snf * 8;                // E columns, F rows, F slots, border partials
        b += (size_t)(p->nblocks + 1) * (6 * 4 + 2 * 8) + 64 * 8;  // per-block tables, one-element minimums
    }
    return b;
}

sdsl_status sdsl_setup(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o,
                       const sdsl_lowrank* lr, const sdsl_allocator* al, void* hip_stream, sdsl_handle* out) {
    if (out) *out = nullptr;
    sdsl_ctx* h = nullptr;
    sdsl_status st = guard(nullptr, [&] {
        if (!out) fail(SDSL_E_INVALID, "null output handle");
        check_partition(A, p, o);
        check_options(o);
        if (al && (!al->alloc) != (!al->free)) fail(SDSL_E_INVALID, "the allocator needs both alloc and free");
        std::unique_ptr<sdsl_ctx> hp(new sdsl_ctx());
        h = hp.get();
        const double t0 = now_ms();
        // Alg. 3 step 1: MC64 on the host; the rest of the setup sees A'
        sdsl_csr Am{};
        std::vector<int64_t> m_rp;
        std::vector<int> m_ci, m_emap;
        std::vector<double> m_val, m_escale, m_rs;
        if (o->mc64) {
            if (lr && lr->k > 0) fail(SDSL_E_INVALID, "MC64 takes no low-rank term");
            if (p->n_border != 0) fail(SDSL_E_INVALID, "MC64 takes no border");
            mc64_transform(A, o->spd != 0, h, m_rp, m_ci, m_val, m_emap, m_escale, m_rs);
            Am = sdsl_csr{A->n, A->nnz, m_rp.data(), m_ci.data(), m_val.data(), SDSL_MEM_HOST};
            A = &Am;
        }
        if (al) h->al = *al;
        h->s = (hipStream_t)hip_stream;
        h->o = *o;
        h->n = A->n;
        h->nnz = A->nnz;
        h->nbd = p->n_border;
        h->n_int = A->n - p->n_border;
        h->nb = p->nblocks;
        h->bp_h.assign(p->block_ptr, p->block_ptr + p->nblocks + 1);
        const int n = h->n;
        const int64_t nnz = h->nnz;
        // row pointer check on the host
        int64_t ends[2];
        if (A->mem == SDSL_MEM_HOST) {
            ends[0] = A->row_ptr[0];
            ends[1] = A->row_ptr[n];
        } else {
            hip_check(hipMemcpy(&ends[0], A->row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost), "copy");
            hip_check(hipMemcpy(&ends[1], A->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost), "copy");
        }
        if (ends[0] != 0 || ends[1] != nnz) fail(SDSL_E_INVALID, "row_ptr must run from 0 to nnz");
        hip_check(hipHostMalloc((void**)&h->st_h, sizeof(KrylovState), hipHostMallocDefault), "pinned alloc");
        hip_check(hipHostMalloc((void**)&h->scal_h, 4 * sizeof(double), hipHostMallocDefault), "pinned alloc");
        hip_check(hipHostMalloc((void**)&h->vout_h, sizeof(ValidateOut), hipHostMallocDefault), "pinned alloc");
        // operator
        int64_t* rp64 = h->alloc<int64_t>(n + 1);
        h->rp = h->alloc<int>(n + 1);
        h->ci = h->alloc<int>(nnz);
        h->v = h->alloc<double>(nnz);
        h->v32 = h->alloc<float>(nnz);
        h->diag = h->alloc<double>(n);
        h->bp = h->alloc<int>(h->nb + 1);
        h->vout = h->alloc<ValidateOut>(1);
        const hipMemcpyKind kind = A->mem == SDSL_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        hip_check(hipMemcpyAsync(rp64, A->row_ptr, (n + 1) * sizeof(int64_t), kind, h->s), "copy");
        hip_check(hipMemcpyAsync(h->ci, A->col, nnz * sizeof(int), kind, h->s), "copy");
        hip_check(hipMemcpyAsync(h->v, A->val, nnz * sizeof(double), kind, h->s), "copy");
        hip_check(hipMemcpyAsync(h->bp, h->bp_h.data(), (h->nb + 1) * sizeof(int), hipMemcpyHostToDevice, h->s),
                  "copy");
        validate_values(h, rp64);
        launch_rowptr32(n, rp64, h->rp, h->s);
        launch_cast_f32(nnz, h->v, h->v32, h->s);
        h->check_launch();
        h->lanes = spmv_lanes((double)nnz / n);
        h->grid = spmv_grid(n);
        // near window of the SpMV: used when at least half of the entries
        // fall inside it (fixed by the pattern)
        {
            unsigned long long* cnt = h->alloc<unsigned long long>(1);
            hip_check(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), h->s), "memset");
            launch_spmv_near(n, h->grid, h->rp, h->ci, kSpmvHalo, cnt, h->s);
            h->check_launch();
            unsigned long long near = 0;
            hip_check(hipMemcpyAsync(&near, cnt, sizeof(near), hipMemcpyDeviceToHost, h->s), "copy");
            h->sync();
            h->halo = 2 * near >= (unsigned long long)nnz ? kSpmvHalo : 0;
        }
        setup_lowrank(h, lr);
        // preconditioner buffers (capacity: every entry of M)
        const int ni = h->n_int;
        if ((int64_t)ni * kBjEllWidth >= (int64_t(1) << 31))
            fail(SDSL_E_INVALID, "block-Jacobi part limited to 2^31 / " + std::to_string(kBjEllWidth) + " rows");
        h->prp = h->alloc<int>(ni + 1);
        h->pci = h->alloc<int>(nnz);
        h->pcap = nnz;
        h->pv_corr = h->alloc<double>(nnz);
        h->pv = h->alloc<double>(nnz);
        h->pdiag = h->alloc<int>(ni);
        h->cnt = h->alloc<int>(ni);
        h->ucnt = h->alloc<int>(ni);
        h->dropsum = h->alloc<double>(ni);
        h->scan_tmp = h->alloc<int>((ni + 1023) / 1024 + 2);
        h->shifts = h->alloc<double>(h->nb);
        h->nfix = h->alloc<int>(1);
        h->bstatus = h->alloc<int>(h->nb);
        h->spin_err = h->alloc<int>(1);
        h->lrp = h->alloc<int>(ni + 1);
        h->urp = h->alloc<int>(ni + 1);
        h->lci = h->alloc<int>(nnz);
        h->uci = h->alloc<int>(nnz);
        h->lval = h->alloc<double>(nnz);
        h->uval = h->alloc<double>(nnz);
        h->udiag = h->alloc<double>(ni);
        h->lch = h->alloc<int2>(ni + h->nb);
        h->uch = h->alloc<int2>(ni + h->nb);
        h->lnl = h->alloc<int>(ni + h->nb);
        h->unl = h->alloc<int>(ni + h->nb);
        h->llev = h->alloc<int>(ni);
        h->ulev = h->alloc<int>(ni);
        h->lval32 = h->alloc<float>(nnz);
        h->uval32 = h->alloc<float>(nnz);
        h->udiag32 = h->alloc<float>(ni);
        h->lell_c = h->alloc<int>((size_t)ni * kBjEllWidth);
        h->uell_c = h->alloc<int>((size_t)ni * kBjEllWidth);
        h->lell_v = h->alloc<double>((size_t)ni * kBjEllWidth);
        h->uell_v = h->alloc<double>((size_t)ni * kBjEllWidth);
        h->lell_v32 = h->alloc<float>((size_t)ni * kBjEllWidth);
        h->uell_v32 = h->alloc<float>((size_t)ni * kBjEllWidth);
        h->lperm = h->alloc<int2>(ni);
        h->uperm = h->alloc<int2>(ni);
        h->lpos = h->alloc<int>(ni);
        h->upos = h->alloc<int>(ni);
        h->lorp = h->alloc<int>(ni + 1);
        h->uorp = h->alloc<int>(ni + 1);
        h->loci = h->alloc<int>(nnz);
        h->uoci = h->alloc<int>(nnz);
        h->lov = h->alloc<double>(nnz);
        h->uov = h->alloc<double>(nnz);
        h->lov32 = h->alloc<float>(nnz);
        h->uov32 = h->alloc<float>(nnz);
        // Krylov workspace
        h->x = h->alloc<double>(n);
        h->r = h->alloc<double>(n);
        h->z = h->alloc<double>(n);
        h->p = h->alloc<double>(n);
        h->q = h->alloc<double>(n);
        h->y = h->alloc<double>(n);
        h->d = h->alloc<double>(n);
        h->rf = h->alloc<double>(n);
        h->xref = h->alloc<double>(n);
        h->x32 = h->alloc<float>(n);
        h->r32 = h->alloc<float>(n);
        h->z32 = h->alloc<float>(n);
        h->p32 = h->alloc<float>(n);
        h->q32 = h->alloc<float>(n);
        h->y32 = h->alloc<float>(n);
        h->part_pq = h->alloc<double>(h->grid);
        h->part_rz = h->alloc<double>(2 * h->nb);
        h->part_rr = h->alloc<double>(h->nb);
        h->part_b = h->alloc<double>(h->grid);
        h->part_res = h->alloc<double>(h->grid);
        h->bi_part = h->alloc<double>((size_t)6 * bicg_grid(n));
        h->scal = h->alloc<double>(4);
        h->st = h->alloc<KrylovState>(1);
        if (o->method == SDSL_BBD) {
            if (lr && lr->k > 0) fail(SDSL_E_INVALID, "the BBD method takes no low-rank term");
            if (h->nbd <= 0) fail(SDSL_E_INVALID, "the BBD method needs a border (n_border > 0)");
            std::vector<int64_t> rph(n + 1);
            std::vector<int> cih(nnz);
            const hipMemcpyKind dk = A->mem == SDSL_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
            hip_check(hipMemcpy(rph.data(), A->row_ptr, (n + 1) * sizeof(int64_t), dk), "copy");
            hip_check(hipMemcpy(cih.data(), A->col, nnz * sizeof(int), dk), "copy");
            setup_bbd(h, rph, cih);
        }
        if (h->mc64) {
            h->m_rowof = h->alloc<int>(n);
            h->m_emap = h->alloc<int>(nnz);
            h->m_rs = h->alloc<double>(n);
            h->m_cs = h->alloc<double>(n);
            h->m_escale = h->alloc<double>(nnz);
            h->m_b = h->alloc<double>(n);
            h->m_y = h->alloc<double>(n);
            const hipMemcpyKind hd = hipMemcpyHostToDevice;
            hip_check(hipMemcpyAsync(h->m_rowof, h->m_rowof_h.data(), n * sizeof(int), hd, h->s), "copy");
            hip_check(hipMemcpyAsync(h->m_emap, m_emap.data(), nnz * sizeof(int), hd, h->s), "copy");
            hip_check(hipMemcpyAsync(h->m_rs, m_rs.data(), n * sizeof(double), hd, h->s), "copy");
            hip_check(hipMemcpyAsync(h->m_cs, h->m_dc_h.data(), n * sizeof(double), hd, h->s), "copy");
            hip_check(hipMemcpyAsync(h->m_escale, m_escale.data(), nnz * sizeof(double), hd, h->s), "copy");
        }
        build_precond(h);
        h->sync();
        h->release(rp64);
        h->info.device_bytes = (int64_t)h->bytes;
        h->info.nnz_dropped = 0;
        h->info.setup_ms = now_ms() - t0;
        *out = hp.release();
    });
    return st;
}

sdsl_status sdsl_refactor(sdsl_handle h, const double* new_val) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!new_val) fail(SDSL_E_INVALID, "null values");
        check_idle(h);
        const double t0 = now_ms();
        check_values(h, new_val);
        take_values(h, new_val);
        launch_cast_f32(h->nnz, h->v, h->v32, h->s);
        h->check_launch();
        build_precond(h);
        h->info.setup_ms = now_ms() - t0;
    });
}

sdsl_status sdsl_update_values(sdsl_handle h, const double* new_val) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!new_val) fail(SDSL_E_INVALID, "null values");
        check_idle(h);
        check_values(h, new_val);
        take_values(h, new_val);
        launch_cast_f32(h->nnz, h->v, h->v32, h->s);
        h->check_launch();
        h->sync();
    });
}

sdsl_status sdsl_set_max_iter(sdsl_handle h, int32_t max_iter) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (max_iter < 1) fail(SDSL_E_INVALID, "max_iter must be positive");
        check_idle(h);
        h->o.max_iter = max_iter;
    });
}

sdsl_status sdsl_solve(sdsl_handle h, const double* b, double* x, double tol, int32_t* iters, double* relres) {
    if (!h) return SDSL_E_INVALID;
    sdsl_status result = SDSL_OK;
    sdsl_status st = guard(h, [&] {
        if (!b || !x) fail(SDSL_E_INVALID, "null vector");
        if (!(tol > 0.0)) fail(SDSL_E_INVALID, "tol must be positive");
        check_idle(h);
        SolveTask t;
        if (h->o.graphs && h->lr.k == 0 && h->bd.k == 0) {
            // iterations through the shared-launch kernels, replayed from a graph
            if (!h->own) h->own = make_own_group(h);
            struct Clear {  // also on an error: nothing of this solve stays queued
                sdsl_ctx* h;
                ~Clear() {
                    h->defer = nullptr;
                    h->own->recs.clear();
                    h->unflushed = false;
                    h->holder = nullptr;
                }
            } clear{h};
            h->defer = h->own;
            t.begin(h, b, x, tol);
            h->own->flush();
            while (!t.finished) {
                t.step();
                h->own->flush();
            }
        } else {
            t.begin(h, b, x, tol);
            while (!t.finished) t.step();
        }
        if (iters) *iters = t.total_its;
        if (relres) *relres = t.relres;
        result = t.status;
    });
    if (st == SDSL_OK && result != SDSL_OK)
        h->err = result == SDSL_E_BREAKDOWN ? "Krylov breakdown" : "tolerance not reached";
    return st != SDSL_OK ? st : result;
}

sdsl_status sdsl_solve_begin(sdsl_handle h, const double* b, double* x, double tol) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!b || !x) fail(SDSL_E_INVALID, "null vector");
        if (!(tol > 0.0)) fail(SDSL_E_INVALID, "tol must be positive");
        check_idle(h);
        if (h->task) delete_task(h->task);
        h->task = new SolveTask();
        h->task->begin(h, b, x, tol);
    });
}

sdsl_status sdsl_solve_step(sdsl_handle h, int32_t* done) {
    if (!h || !done) return SDSL_E_INVALID;
    *done = 0;
    return guard(h, [&] {
        if (!h->task) fail(SDSL_E_STATE, "no solve was begun on this handle");
        if (h->unflushed) fail(SDSL_E_STATE, "the solve's first iterations wait for its group's next step");
        SolveTask& t = *h->task;
        if (!t.finished) {
            const hipError_t q = hipStreamQuery(h->s);
            if (q == hipErrorNotReady) return;  // its launches are still running
            if (q != hipSuccess) hip_check(q, "stream query");
            t.step();
        }
        *done = t.finished ? 1 : 0;
    });
}

sdsl_status sdsl_solve_end(sdsl_handle h, int32_t* iters, double* relres) {
    if (!h) return SDSL_E_INVALID;
    sdsl_status result = SDSL_OK;
    sdsl_status st = guard(h, [&] {
        if (!h->task || !h->task->finished) fail(SDSL_E_STATE, "the solve has not finished");
        if (iters) *iters = h->task->total_its;
        if (relres) *relres = h->task->relres;
        result = h->task->status;
        delete_task(h->task);
        h->task = nullptr;
    });
    if (st == SDSL_OK && result != SDSL_OK)
        h->err = result == SDSL_E_BREAKDOWN ? "Krylov breakdown" : "tolerance not reached";
    return st != SDSL_OK ? st : result;
}

sdsl_status sdsl_solve_batch(int32_t k, const sdsl_handle* hs, const double* const* b, double* const* x,
                             double tol, int32_t* iters, double* relres) {
    if (k < 0 || (k > 0 && (!hs || !b || !x || !iters || !relres))) return SDSL_E_INVALID;
    std::vector<SolveTask> tasks(k);
    std::vector<sdsl_status> res(k, SDSL_OK);
    std::vector<bool> live(k, false);
    for (int i = 0; i < k; ++i) {
        if (!hs[i]) { res[i] = SDSL_E_INVALID; continue; }
        res[i] = guard(hs[i], [&] {
            if (!b[i] || !x[i]) fail(SDSL_E_INVALID, "null vector");
            if (!(tol > 0.0)) fail(SDSL_E_INVALID, "tol must be positive");
            for (int j = 0; j < i; ++j)
                if (hs[j] == hs[i]) fail(SDSL_E_STATE, "the same handle appears twice in one batch");
            check_idle(hs[i]);
            tasks[i].begin(hs[i], b[i], x[i], tol);
        });
        live[i] = res[i] == SDSL_OK;
    }
    bool any = true;
    while (any) {
        any = false;
        for (int i = 0; i < k; ++i) {
            if (!live[i]) continue;
            if (tasks[i].finished) { live[i] = false; continue; }
            any = true;
            res[i] = guard(hs[i], [&] { tasks[i].step(); });
            if (res[i] != SDSL_OK) live[i] = false;
        }
    }
    sdsl_status first = SDSL_OK;
    for (int i = 0; i < k; ++i) {
        if (res[i] == SDSL_OK && tasks[i].finished) res[i] = tasks[i].status;
        iters[i] = tasks[i].total_its;
        relres[i] = tasks[i].relres;
        if (first == SDSL_OK && res[i] != SDSL_OK) first = res[i];
    }
    return first;
}

sdsl_status sdsl_group_create(void* hip_stream, int32_t use_graphs, const sdsl_allocator* al, sdsl_group* out) {
    if (!out) return SDSL_E_INVALID;
    *out = nullptr;
    if (al && (!al->alloc) != (!al->free)) return SDSL_E_INVALID;
    sdsl_group g = nullptr;
    sdsl_status st = guard(nullptr, [&] {
        g = new sdsl_group_s();
        g->s = (hipStream_t)hip_stream;
        g->graphs = use_graphs != 0;
        if (al) g->al = *al;
        hip_check(hipEventCreateWithFlags(&g->copied, hipEventDisableTiming), "event create");
        if (g->graphs) hip_check(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking), "stream create");
    });
    if (st != SDSL_OK) {
        delete g;
        return st;
    }
    *out = g;
    return SDSL_OK;
}

sdsl_status sdsl_group_begin(sdsl_group g, sdsl_handle h, const double* b, double* x, double tol) {
    if (!g || !h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!b || !x) fail(SDSL_E_INVALID, "null vector");
        if (!(tol > 0.0)) fail(SDSL_E_INVALID, "tol must be positive");
        if (h->s != g->s) fail(SDSL_E_INVALID, "the handle runs on another stream than the group");
        check_idle(h);
        if (h->task) delete_task(h->task);
        h->task = new SolveTask();
        h->defer = g;
        try {
            h->task->begin(h, b, x, tol);
        } catch (...) {
            h->defer = nullptr;
            throw;
        }
        h->defer = nullptr;
    });
}

sdsl_status sdsl_group_step(sdsl_group g, int32_t k, const sdsl_handle* hs, int32_t* done) {
    if (!g || k < 0 || (k > 0 && (!hs || !done))) return SDSL_E_INVALID;
    sdsl_status first = SDSL_OK;
    for (int i = 0; i < k; ++i) {
        done[i] = 0;
        sdsl_handle h = hs[i];
        if (!h) {
            if (first == SDSL_OK) first = SDSL_E_INVALID;
            continue;
        }
        const sdsl_status st = guard(h, [&] {
            for (int j = 0; j < i; ++j)
                if (hs[j] == h) fail(SDSL_E_STATE, "the same handle appears twice in one group step");
            if (h->s != g->s) fail(SDSL_E_INVALID, "the handle runs on another stream than the group");
            if (!h->task) fail(SDSL_E_STATE, "no solve was begun on this handle");
            SolveTask& t = *h->task;
            // iterations collected by sdsl_group_begin go out with this step's
            if (!t.finished && !h->unflushed) {
                h->defer = g;
                try {
                    t.step();
                } catch (...) {
                    h->defer = nullptr;
                    throw;
                }
                h->defer = nullptr;
            }
            done[i] = t.finished ? 1 : 0;
        });
        if (st != SDSL_OK && first == SDSL_OK) first = st;
    }
    const sdsl_status fs = guard(nullptr, [&] { g->flush(); });
    return first != SDSL_OK ? first : fs;
}

sdsl_status sdsl_group_get_stats(sdsl_group g, sdsl_group_stats* out) {
    if (!g || !out) return SDSL_E_INVALID;
    *out = g->stats;
    return SDSL_OK;
}

void sdsl_group_destroy(sdsl_group g) {
    if (!g) return;
    (void)guard(nullptr, [&] { g->flush(); });
    delete g;
}

sdsl_status sdsl_get_info(sdsl_handle h, sdsl_info* out) {
    if (!h || !out) return SDSL_E_INVALID;
    *out = h->info;
    out->device_bytes = (int64_t)h->bytes;
    return SDSL_OK;
}

const char* sdsl_last_error(sdsl_handle h) { return h ? h->err.c_str() : g_thread_err.c_str(); }

void sdsl_destroy(sdsl_handle h) {
    if (!h) return;
    if (h->unflushed && h->holder) {
        // iterations a group still holds for this handle are dropped
        auto& v = h->holder->recs;
        v.erase(std::remove_if(v.begin(), v.end(), [&](const IssueRec& r) { return r.h == h; }), v.end());
    }
    delete h;
}

sdsl_status sdsl_spmv(sdsl_handle h, int32_t prec, const void* x, void* y) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!x || !y) fail(SDSL_E_INVALID, "null vector");
        check_idle(h);
        const CsrView A{h->n, h->rp, h->ci, h->halo};
        if (prec == SDSL_FP64) {
            apply_op64(h, (const double*)x, (double*)y);
        } else {
            if (h->lr.k > 0) launch_lowrank_tdot<float>(h->lr, (const float*)x, nullptr, LR_SCALED, h->s);
            launch_spmv<float, float>(A, h->v32, h->lr, (const float*)x, (float*)y, nullptr, nullptr, h->lanes,
                                      h->grid, h->s);
        }
        h->check_launch();
        h->sync();
    });
}

sdsl_status sdsl_precond_apply(sdsl_handle h, int32_t prec, const void* r, void* z) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!r || !z) fail(SDSL_E_INVALID, "null vector");
        check_idle(h);
        PcgVecs V{};
        V.r = const_cast<void*>(r);
        V.z = z;
        hip_check(hipMemsetAsync(h->spin_err, 0, sizeof(int), h->s), "memset");
        if (prec == SDSL_FP64) {
            apply_prec64(h, (const double*)r, (double*)z);
        } else {
            V.y = h->y32;
            launch_bj<float, float>(0, bj_dev(h, true), V, nullptr, 0, h->s);
            if (h->bd.k > 0) {
                launch_lowrank_tdot<float>(h->lr, (const float*)z, nullptr, LR_BORDER, h->s);
                launch_border_fix<float>(h->n, (float*)z, h->bd, h->s);
            }
        }
        h->check_launch();
        h->sync();
    });
}

sdsl_status sdsl_residual(sdsl_handle h, const double* b, const double* x, double* r, double* norm) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!b || !x || !r) fail(SDSL_E_INVALID, "null vector");
        check_idle(h);
        const double nr = true_residual(h, b, x, r);
        if (norm) *norm = nr;
    });
}

sdsl_status sdsl_residual_noalloc(sdsl_handle h, const double* b, const double* x, double* r, double* norm) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!b || !x || !r) fail(SDSL_E_INVALID, "null vector");
        check_idle(h);
        // scratch layout: [0] = ||r||^2, [1, 1 + grid) = per-workgroup
        // partials of ||r||^2, then the compensated U^T x slice sums of the
        // low-rank term (2 k slices); every entry is written before it is read
        const size_t lr_part = h->lr.k > 0 ? (size_t)2 * h->lr.k * h->lr.slices : 0;
        const size_t need = 1 + (size_t)h->grid + lr_part;
        if (need > kNoAllocDoubles)
            fail(SDSL_E_INVALID, "the allocation-free residual needs " + std::to_string(need) +
                                     " scratch doubles for this system; the limit is " +
                                     std::to_string(kNoAllocDoubles) + " (about 8M rows)");
        double* s = scratch_here();
        LowRankDev lr = h->lr;
        lr.part = s + 1 + h->grid;
        const CsrView A{h->n, h->rp, h->ci, h->halo};
        launch_residual(A, h->v, lr, b, x, r, s + 1, h->lanes, h->grid, h->s);
        launch_sum_partials(s + 1, h->grid, s, h->s);
        h->check_launch();
        hip_check(hipMemcpyAsync(h->scal_h + 3, s, sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
        h->sync();
        if (norm) *norm = std::sqrt(h->scal_h[3]);
    });
}

sdsl_status sdsl_get_factors(sdsl_handle h, int64_t* row_ptr, int32_t* col, double* corrected, double* lu,
                             double* shifts) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        h->sync();
        if (row_ptr) {
            std::vector<int> tmp(h->n_int + 1);
            hip_check(hipMemcpy(tmp.data(), h->prp, (h->n_int + 1) * sizeof(int), hipMemcpyDeviceToHost), "copy");
            for (int i = 0; i <= h->n_int; ++i) row_ptr[i] = tmp[i];
        }
        const size_t m = (size_t)h->p_nnz;
        if (col) hip_check(hipMemcpy(col, h->pci, m * sizeof(int), hipMemcpyDeviceToHost), "copy");
        if (corrected) hip_check(hipMemcpy(corrected, h->pv_corr, m * sizeof(double), hipMemcpyDeviceToHost), "copy");
        if (lu) hip_check(hipMemcpy(lu, h->pv, m * sizeof(double), hipMemcpyDeviceToHost), "copy");
        if (shifts) hip_check(hipMemcpy(shifts, h->shifts, h->nb * sizeof(double), hipMemcpyDeviceToHost), "copy");
    });
}

sdsl_status sdsl_get_mc64(sdsl_handle h, int32_t* row_of, double* row_scale, double* col_scale) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!h->mc64) fail(SDSL_E_STATE, "the handle was set up without MC64");
        const size_t n = (size_t)h->n;
        if (row_of) std::copy(h->m_rowof_h.begin(), h->m_rowof_h.end(), row_of);
        if (row_scale) std::copy(h->m_dr_h.begin(), h->m_dr_h.begin() + n, row_scale);
        if (col_scale) std::copy(h->m_dc_h.begin(), h->m_dc_h.begin() + n, col_scale);
    });
}

sdsl_status sdsl_get_schur(sdsl_handle h, double* lu, int32_t* piv, double* inv) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!h->bbd) fail(SDSL_E_STATE, "not a BBD handle");
        h->sync();
        const size_t m = (size_t)h->nbd * h->nbd;
        if (lu) hip_check(hipMemcpy(lu, h->bbd_S, m * sizeof(double), hipMemcpyDeviceToHost), "copy");
        if (piv) hip_check(hipMemcpy(piv, h->bbd_piv, h->nbd * sizeof(int), hipMemcpyDeviceToHost), "copy");
        if (inv) hip_check(hipMemcpy(inv, h->bbd_Sinv, m * sizeof(double), hipMemcpyDeviceToHost), "copy");
    });
}

}  // extern "C"
