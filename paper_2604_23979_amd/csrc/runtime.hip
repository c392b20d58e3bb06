// Host runtime and C ABI of the solver: the handle, preconditioner setup and
// refactorisation, and the Krylov drivers (PCG in FP64, FP32-inner PCG inside
// FP64 iterative refinement).  Every numerical step runs in the gfx950
// kernels; the host only sequences launches and reads a few scalars.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <string>
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
struct sdsl_ctx {
    hipStream_t s = nullptr;
    sdsl_options o{};
    int n = 0, n_int = 0, nbd = 0, nb = 0;
    int64_t nnz = 0;
    std::vector<int> bp_h;
    std::vector<void*> allocs;
    size_t bytes = 0;
    std::string err;

    // operator
    int *bp = nullptr, *rp = nullptr, *ci = nullptr;
    double* v = nullptr;
    float* v32 = nullptr;
    double* diag = nullptr;
    int lanes = 4, grid = 8;
    // low-rank term
    LowRankDev lr64{}, lr32{};
    // block-Jacobi preconditioner
    int *prp = nullptr, *pci = nullptr, *pdiag = nullptr, *cnt = nullptr, *scan_tmp = nullptr;
    double *pv_corr = nullptr, *pv = nullptr, *dropsum = nullptr, *shifts = nullptr;
    float* pv32 = nullptr;
    int *nfix = nullptr, *bstatus = nullptr, *spin_err = nullptr;
    int p_nnz = 0;
    // Krylov workspace
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *y = nullptr, *d = nullptr;
    double* rf = nullptr;  // right-hand side of an FP64 fallback solve
    float *x32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *y32 = nullptr;
    double *part_pq = nullptr, *part_rz = nullptr, *part_rr = nullptr, *part_b = nullptr, *part_res = nullptr;
    double* scal = nullptr;  // [0] = ||r||^2 of the latest residual, [1] = ||b||^2
    KrylovState* st = nullptr;
    KrylovState* st_h = nullptr;  // pinned
    double* scal_h = nullptr;     // pinned
    ValidateOut* vout = nullptr;
    ValidateOut* vout_h = nullptr;
    sdsl_info info{};

    template <typename T>
    T* alloc(size_t count) {
        void* ptr = nullptr;
        const size_t b = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&ptr, b) != hipSuccess) {
            (void)hipGetLastError();
            fail(SDSL_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
        }
        allocs.push_back(ptr);
        bytes += b;
        return (T*)ptr;
    }
    ~sdsl_ctx() {
        if (s) (void)hipStreamSynchronize(s);
        for (void* a : allocs) (void)hipFree(a);
        if (st_h) (void)hipHostFree(st_h);
        if (scal_h) (void)hipHostFree(scal_h);
        if (vout_h) (void)hipHostFree(vout_h);
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
void check_values(sdsl_ctx* h, const double* vals) {
    launch_count_nonfinite(h->nnz, vals, h->vout, h->s);
    h->check_launch();
    hip_check(hipMemcpyAsync(h->vout_h, h->vout, sizeof(ValidateOut), hipMemcpyDeviceToHost, h->s), "copy");
    h->sync();
    if (h->vout_h->nonfinite) fail(SDSL_E_INVALID, "non-finite matrix values");
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
    hip_check(hipMemsetAsync(h->nfix, 0, sizeof(int), s), "memset");
    hip_check(hipMemsetAsync(h->spin_err, 0, sizeof(int), s), "memset");
    launch_ilu0(h->nb, h->bp, h->prp, h->pci, h->pv_corr, h->pv, h->pdiag, h->o.spd, h->o.pivot, h->o.shift0,
                h->shifts, h->nfix, h->bstatus, h->spin_err, s);
    h->check_launch();
    int kept = 0, nfix = 0, spin = 0;
    hip_check(hipMemcpyAsync(&kept, h->prp + h->n_int, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(&nfix, h->nfix, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(&spin, h->spin_err, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    std::vector<int> bst(h->nb);
    std::vector<double> sh(h->nb);
    hip_check(hipMemcpyAsync(bst.data(), h->bstatus, h->nb * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipMemcpyAsync(sh.data(), h->shifts, h->nb * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    h->sync();
    h->p_nnz = kept;
    launch_cast_f32(kept, h->pv, h->pv32, s);
    h->check_launch();
    h->info.nnz_kept = kept;
    int64_t in_block = 0;
    (void)in_block;
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
    h->info.setup_ms = now_ms() - t0;
    // algorithmic bytes of one FP64 PCG iteration (SpMV + BJ apply + vectors)
    const int64_t n = h->n;
    h->info.bytes_per_iter = (8 + 4) * h->nnz + (4 + 16) * n + (8 + 4) * (int64_t)kept + (8 + 32) * n + 72 * n;
}

void setup_lowrank(sdsl_ctx* h, const sdsl_lowrank* lr) {
    if (!lr || lr->k <= 0) return;
    const int k = lr->k, n = h->n;
    if (k > 64) fail(SDSL_E_INVALID, "low-rank term limited to 64 columns");
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
        if (!std::isfinite(cj)) fail(SDSL_E_INVALID, "non-finite low-rank scale");
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
    int* d_urp = h->alloc<int>(n + 1);
    int* d_uci = h->alloc<int>(m);
    double* d_uv = h->alloc<double>(m);
    float* d_uv32 = h->alloc<float>(m);
    int* d_ucp = h->alloc<int>(k + 1);
    int* d_uri = h->alloc<int>(m);
    double* d_ucv = h->alloc<double>(m);
    float* d_ucv32 = h->alloc<float>(m);
    double* d_c = h->alloc<double>(k);
    float* d_c32 = h->alloc<float>(k);
    const int slices = 32;
    double* part = h->alloc<double>(2 * k * slices);
    std::vector<float> f(m);
    hip_check(hipMemcpy(d_urp, urp32.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_uci, uci.data(), m * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_uv, uv.data(), m * sizeof(double), hipMemcpyHostToDevice), "copy");
    for (int64_t p = 0; p < m; ++p) f[p] = (float)uv[p];
    hip_check(hipMemcpy(d_uv32, f.data(), m * sizeof(float), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_ucp, cp.data(), (k + 1) * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_uri, ri.data(), m * sizeof(int), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_ucv, cv.data(), m * sizeof(double), hipMemcpyHostToDevice), "copy");
    for (int64_t p = 0; p < m; ++p) f[p] = (float)cv[p];
    hip_check(hipMemcpy(d_ucv32, f.data(), m * sizeof(float), hipMemcpyHostToDevice), "copy");
    hip_check(hipMemcpy(d_c, c.data(), k * sizeof(double), hipMemcpyHostToDevice), "copy");
    std::vector<float> c32(k);
    for (int j = 0; j < k; ++j) c32[j] = (float)c[j];
    hip_check(hipMemcpy(d_c32, c32.data(), k * sizeof(float), hipMemcpyHostToDevice), "copy");
    LowRankDev base;
    base.k = k;
    base.slices = slices;
    base.urp = d_urp;
    base.uci = d_uci;
    base.ucp = d_ucp;
    base.uri = d_uri;
    base.part = part;
    h->lr64 = base;
    h->lr64.uv = d_uv;
    h->lr64.ucv = d_ucv;
    h->lr64.c = d_c;
    h->lr32 = base;
    h->lr32.uv = d_uv32;
    h->lr32.ucv = d_ucv32;
    h->lr32.c = d_c32;
}

BJDev bj_dev(sdsl_ctx* h, bool fp32) {
    BJDev P;
    P.nblocks = h->nb;
    P.bp = h->bp;
    P.prp = h->prp;
    P.pci = h->pci;
    P.pv = fp32 ? (const void*)h->pv32 : (const void*)h->pv;
    P.pdiag = h->pdiag;
    return P;
}

// ------------------------------------------------------------- PCG engine
// One PCG run on the device.  The right-hand side is already in r and x is
// zero; `issue` launches up to `count` iterations (kernels become no-ops once
// the device state says done); `poll` synchronises and reads that state.
template <typename T>
struct Pcg {
    sdsl_ctx* h;
    T *x, *r, *z, *p, *q, *y;
    const T* v;
    const LowRankDev* lr;
    BJDev P;
    PcgVecs V;
    int it = 0;      // next iteration index
    int done_its = 0;

    void init(bool fp32) {
        P = bj_dev(h, fp32);
        V.x = x; V.r = r; V.p = p; V.q = q; V.z = z; V.y = y;
        V.part_pq = h->part_pq;
        V.npq = h->grid;
        V.part_rz = h->part_rz;
        V.part_rr = h->part_rr;
    }
    // z = P^{-1} r, p = z, (r,z) into the parity slot of iteration it-1
    void start() {
        launch_bj<T>(2, P, V, h->st, it - 1, h->s);
        launch_copy<T>(h->n, z, p, h->s);
        if (lr->k > 0) launch_lowrank_tdot<T>(*lr, p, h->st, h->s);
        h->check_launch();
    }
    void issue(int count) {
        const CsrView A{h->n, h->rp, h->ci};
        for (int k = 0; k < count; ++k, ++it) {
            launch_spmv<T>(A, v, *lr, p, q, h->part_pq, h->st, h->lanes, h->grid, h->s);
            launch_bj<T>(1, P, V, h->st, it, h->s);
            launch_pcg_pupdate<T>(h->n, V, h->nb, h->st, it, h->s);
            if (lr->k > 0) launch_lowrank_tdot<T>(*lr, p, h->st, h->s);
        }
        h->check_launch();
    }
    const KrylovState& poll() {
        hip_check(hipMemcpyAsync(h->st_h, h->st, sizeof(KrylovState), hipMemcpyDeviceToHost, h->s), "copy");
        h->sync();
        if (h->st_h->spin_err) fail(SDSL_E_DEVICE, "triangular solve in-workgroup wait limit exceeded");
        return *h->st_h;
    }
};

// sum of a device partial array into scal[idx], then copied to the host
double reduce_to_host(sdsl_ctx* h, const double* part, int m, int idx) {
    launch_sum_partials(part, m, h->scal + idx, h->s);
    h->check_launch();
    hip_check(hipMemcpyAsync(h->scal_h + idx, h->scal + idx, sizeof(double), hipMemcpyDeviceToHost, h->s), "copy");
    h->sync();
    return h->scal_h[idx];
}

double true_residual(sdsl_ctx* h, const double* b, const double* x, double* r) {
    const CsrView A{h->n, h->rp, h->ci};
    launch_residual(A, h->v, h->lr64, b, x, r, h->part_res, h->lanes, h->grid, h->s);
    h->check_launch();
    return std::sqrt(reduce_to_host(h, h->part_res, h->grid, 0));
}

// ------------------------------------------------------------- solve task
// Resumable solve: `step()` issues the next stretch of device work and
// returns; `wait()` synchronises on it.  sdsl_solve runs one task to the end;
// sdsl_solve_batch interleaves several on their own streams.
struct SolveTask {
    sdsl_ctx* h = nullptr;
    const double* b = nullptr;
    double* xout = nullptr;
    double tol = 1e-8;
    double nb = 0.0;
    int total_its = 0, outer = 0, fallbacks = 0, restarts = 0;
    double relres = 1.0;
    sdsl_status status = SDSL_OK;
    bool finished = false;
    double t0 = 0.0;

    enum Phase { P64_ITER, IR_ITER } phase = P64_ITER;
    // FP64 PCG (also the IR fallback)
    Pcg<double> pcg64{};
    double* pcg_rhs = nullptr;   // b (plain solve) or the IR residual (fallback)
    double* pcg_out = nullptr;   // x (plain) or d (fallback)
    double pcg_tol = 0.0;
    bool fallback = false;
    // FP32 inner PCG
    Pcg<float> pcg32{};
    double nr = 0.0, prev = 0.0;
    int slow = 0;

    void begin(sdsl_ctx* hh, const double* bb, double* xx, double tt) {
        h = hh; b = bb; xout = xx; tol = tt;
        t0 = now_ms();
        launch_sqnorm_partials(h->n, b, h->part_b, h->grid, h->s);
        h->check_launch();
        nb = std::sqrt(reduce_to_host(h, h->part_b, h->grid, 1));
        launch_fill<double>(h->n, xout, 0.0, h->s);
        if (nb == 0.0) { finish(SDSL_OK, 0.0); return; }
        pcg64 = Pcg<double>{h, h->x, h->r, h->z, h->p, h->q, h->y, h->v, &h->lr64};
        pcg64.init(false);
        pcg32 = Pcg<float>{h, h->x32, h->r32, h->z32, h->p32, h->q32, h->y32, h->v32, &h->lr32};
        pcg32.init(true);
        if (h->o.precision == SDSL_FP64) {
            start_pcg64(b, xout, tol);
        } else {
            phase = IR_ITER;
            ir_outer_check(true);
        }
    }
    // plain FP64 PCG on M out = rhs (x0 = 0) to ||rhs - M out|| <= t ||rhs||
    void start_pcg64(const double* rhs, double* out, double t) {
        phase = P64_ITER;
        pcg_rhs = const_cast<double*>(rhs);
        pcg_out = out;
        pcg_tol = t;
        pcg64.x = out;
        pcg64.V.x = out;
        pcg64.it = 0;
        launch_fill<double>(h->n, out, 0.0, h->s);
        launch_copy<double>(h->n, rhs, h->r, h->s);
        launch_sqnorm_partials(h->n, rhs, h->part_res, h->grid, h->s);
        launch_init_state(h->st, h->part_res, h->grid, t, h->s);
        pcg64.start();
        pcg64.issue(std::min(h->o.check_every, h->o.max_iter - total_its));
    }
    void finish(sdsl_status s, double rr) {
        status = s;
        relres = rr;
        finished = true;
        h->info.solve_ms = now_ms() - t0;
        h->info.relres = rr;
        h->info.inner_iters = total_its;
        h->info.outer_iters = outer;
        h->info.fp64_fallbacks = fallbacks;
        h->info.restarts = restarts;
    }
    // IR: residual of the current x; decide to stop, fall back or run an inner solve
    void ir_outer_check(bool first) {
        if (first) {
            nr = true_residual(h, b, xout, h->r);
        }
        if (nr <= tol * nb) { finish(SDSL_OK, nr / nb); return; }
        if (outer >= h->o.max_outer || total_its >= h->o.max_iter) {
            finish(SDSL_E_NOT_CONVERGED, nr / nb);
            return;
        }
        if (slow >= 2) {
            // FP64 fallback on M d = r for the rest of the tolerance
            fallback = true;
            fallbacks++;
            outer++;
            launch_copy<double>(h->n, h->r, h->rf, h->s);
            start_pcg64(h->rf, h->d, tol * nb / nr);
            return;
        }
        // inner FP32 solve of M d = r / ||r||
        launch_ir_scale_cast(h->n, h->r, h->scal + 0, h->r32, h->s);
        launch_fill<float>(h->n, h->x32, 0.0f, h->s);
        // ||rs||^2 accumulated in FP64 from the FP32 values
        launch_inner_bb();
        launch_init_state(h->st, h->part_res, h->grid, h->o.inner_tol, h->s);
        pcg32.it = 0;
        pcg32.start();
        pcg32.issue(std::min(h->o.check_every, h->o.max_iter - total_its));
    }
    void launch_inner_bb();

    // advance after the pending work finished; returns false once finished
    void step() {
        if (finished) return;
        if (phase == P64_ITER) {
            const KrylovState& s = pcg64.poll();
            if (!s.done) {
                const int used = pcg64.it;
                if (total_its + used >= h->o.max_iter) {
                    total_its += used;
                    double rr = true_residual(h, pcg_rhs, pcg_out, h->r);
                    end_pcg64(SDSL_E_NOT_CONVERGED, rr);
                    return;
                }
                pcg64.issue(std::min(h->o.check_every, h->o.max_iter - total_its - used));
                return;
            }
            const int its = s.iters;
            if (s.breakdown) {
                total_its += its;
                double rr = true_residual(h, pcg_rhs, pcg_out, h->r);
                end_pcg64(SDSL_E_BREAKDOWN, rr);
                return;
            }
            // converged on the recurrence: check the true residual
            const double rr = true_residual(h, pcg_rhs, pcg_out, h->r);
            const double nrhs = fallback ? nr : nb;
            if (rr <= pcg_tol * nrhs || total_its + its >= h->o.max_iter) {
                total_its += its;
                end_pcg64(rr <= pcg_tol * nrhs ? SDSL_OK : SDSL_E_NOT_CONVERGED, rr);
                return;
            }
            // restart from the true residual (now in r); x keeps accumulating
            restarts++;
            total_its += its;
            pcg64.it = 0;
            if (fallback) {
                // bb is ||rhs||^2 of the fallback system
                launch_sqnorm_partials(h->n, pcg_rhs, h->part_res, h->grid, h->s);
                launch_init_state(h->st, h->part_res, h->grid, pcg_tol, h->s);
            } else {
                launch_init_state(h->st, h->part_b, h->grid, pcg_tol, h->s);
            }
            pcg64.start();
            pcg64.issue(std::min(h->o.check_every, h->o.max_iter - total_its));
            return;
        }
        // IR inner FP32 PCG
        const KrylovState& s = pcg32.poll();
        if (!s.done && total_its + pcg32.it < h->o.max_iter) {
            pcg32.issue(std::min(h->o.check_every, h->o.max_iter - total_its - pcg32.it));
            return;
        }
        total_its += s.done ? s.iters : pcg32.it;
        if (s.done && s.breakdown && s.iters == 0) {
            // no progress possible in FP32: force the FP64 fallback
            slow = 2;
        }
        // x += ||r|| d
        launch_ir_update(h->n, xout, h->scal + 0, h->x32, h->s);
        h->check_launch();
        outer++;
        prev = nr;
        nr = true_residual(h, b, xout, h->r);
        slow = (nr > 0.5 * prev) ? slow + 1 : (slow >= 2 ? slow : 0);
        ir_outer_check(false);
    }
    void end_pcg64(sdsl_status st, double rr) {
        if (!fallback) {
            finish(st, rr / nb);
            return;
        }
        // fallback finished: x += d, back to the refinement loop
        fallback = false;
        phase = IR_ITER;
        launch_axpy_x();
        prev = nr;
        nr = true_residual(h, b, xout, h->r);
        slow = 0;
        if (st == SDSL_E_BREAKDOWN) { finish(st, nr / nb); return; }
        ir_outer_check(false);
    }
    void launch_axpy_x();
};

}  // namespace

// small device helpers used by the task (defined here to keep them local)
__global__ void k_axpy1(int n, double* __restrict__ x, const double* __restrict__ d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = x[i] + d[i];
}
__global__ __launch_bounds__(256) void k_sqnorm_f32(int n, const float* __restrict__ a, double* __restrict__ part) {
    __shared__ double red[8];
    const int g = gridDim.x;
    const int per = (n + g - 1) / g;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double s = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) s += (double)a[i] * (double)a[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void SolveTask::launch_axpy_x() {
    const int g = std::min(4096, (h->n + 255) / 256);
    k_axpy1<<<std::max(g, 1), 256, 0, h->s>>>(h->n, xout, h->d);
    h->check_launch();
}
void SolveTask::launch_inner_bb() {
    k_sqnorm_f32<<<h->grid, 256, 0, h->s>>>(h->n, h->r32, h->part_res);
    h->check_launch();
}

namespace {
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

void check_options(const sdsl_options* o) {
    if (o->method != SDSL_BJ && o->method != SDSL_BBD) fail(SDSL_E_INVALID, "unknown method");
    if (o->method == SDSL_BBD) fail(SDSL_E_INVALID, "the BBD method is not available in this library");
    if (o->filter < SDSL_FILTER_NONE || o->filter > SDSL_FILTER_GEOMEAN) fail(SDSL_E_INVALID, "unknown filter");
    if (!(o->tau >= 0.0)) fail(SDSL_E_INVALID, "tau must be >= 0");
    if (!(o->delta >= 0.0) || !std::isfinite(o->delta)) fail(SDSL_E_INVALID, "delta must be finite and >= 0");
    if (o->pivot < SDSL_PIVOT_FAIL || o->pivot > SDSL_PIVOT_SHIFT) fail(SDSL_E_INVALID, "unknown pivot policy");
    if (o->pivot == SDSL_PIVOT_SHIFT && !(o->shift0 > 0.0 && std::isfinite(o->shift0)))
        fail(SDSL_E_INVALID, "shift0 must be positive");
    if (o->krylov != SDSL_PCG) fail(SDSL_E_INVALID, "only PCG is available in this library");
    if (o->max_iter < 1 || o->check_every < 1) fail(SDSL_E_INVALID, "max_iter and check_every must be >= 1");
    if (o->precision != SDSL_FP64 && o->precision != SDSL_FP32_IR) fail(SDSL_E_INVALID, "unknown precision");
    if (o->precision == SDSL_FP32_IR && (!(o->inner_tol > 0.0 && o->inner_tol < 1.0) || o->max_outer < 1))
        fail(SDSL_E_INVALID, "inner_tol must be in (0,1) and max_outer >= 1");
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
}

size_t sdsl_footprint_bytes(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o,
                            const sdsl_lowrank* lr) {
    if (!A || !p || !o || A->n <= 0 || A->nnz < 0) return 0;
    const size_t n = (size_t)A->n, nnz = (size_t)A->nnz, nb = (size_t)std::max(p->nblocks, 1);
    size_t b = 0;
    b += (n + 1) * 4 + nnz * (4 + 8 + 4) + n * 8;           // operator + FP32 copy + diag
    b += (n + 1) * 4 + nnz * (4 + 8 + 8 + 4) + n * (4 + 4 + 8);  // preconditioner capacity
    b += n * (7 * 8 + 6 * 4);                                  // Krylov vectors
    b += (nb + 1) * 4 + nb * (8 + 4) + 2048 * 8 * 4 + nb * 8 * 3;
    if (lr && lr->k > 0) b += (size_t)lr->U.nnz * 2 * (4 + 8 + 4) + (n + 1) * 4;
    b += (n + 1023) / 1024 * 4 + 4096;
    return b;
}

sdsl_status sdsl_setup(const sdsl_csr* A, const sdsl_partition* p, const sdsl_options* o,
                       const sdsl_lowrank* lr, void* hip_stream, sdsl_handle* out) {
    if (out) *out = nullptr;
    sdsl_ctx* h = nullptr;
    sdsl_status st = guard(nullptr, [&] {
        if (!out) fail(SDSL_E_INVALID, "null output handle");
        check_partition(A, p, o);
        check_options(o);
        std::unique_ptr<sdsl_ctx> hp(new sdsl_ctx());
        h = hp.get();
        const double t0 = now_ms();
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
        setup_lowrank(h, lr);
        // preconditioner buffers (capacity: every entry of M)
        h->prp = h->alloc<int>(h->n_int + 1);
        h->pci = h->alloc<int>(nnz);
        h->pv_corr = h->alloc<double>(nnz);
        h->pv = h->alloc<double>(nnz);
        h->pv32 = h->alloc<float>(nnz);
        h->pdiag = h->alloc<int>(h->n_int);
        h->cnt = h->alloc<int>(h->n_int);
        h->dropsum = h->alloc<double>(h->n_int);
        h->scan_tmp = h->alloc<int>((h->n_int + 1023) / 1024 + 2);
        h->shifts = h->alloc<double>(h->nb);
        h->nfix = h->alloc<int>(1);
        h->bstatus = h->alloc<int>(h->nb);
        h->spin_err = h->alloc<int>(1);
        // Krylov workspace
        h->x = h->alloc<double>(n);
        h->r = h->alloc<double>(n);
        h->z = h->alloc<double>(n);
        h->p = h->alloc<double>(n);
        h->q = h->alloc<double>(n);
        h->y = h->alloc<double>(n);
        h->d = h->alloc<double>(n);
        h->rf = h->alloc<double>(n);
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
        h->scal = h->alloc<double>(4);
        h->st = h->alloc<KrylovState>(1);
        build_precond(h);
        h->sync();
        hip_check(hipFree(rp64), "free");
        h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void*)rp64));
        h->bytes -= (size_t)(n + 1) * sizeof(int64_t);
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
        const double t0 = now_ms();
        check_values(h, new_val);
        hip_check(hipMemcpyAsync(h->v, new_val, h->nnz * sizeof(double), hipMemcpyDeviceToDevice, h->s), "copy");
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
        check_values(h, new_val);
        hip_check(hipMemcpyAsync(h->v, new_val, h->nnz * sizeof(double), hipMemcpyDeviceToDevice, h->s), "copy");
        launch_cast_f32(h->nnz, h->v, h->v32, h->s);
        h->check_launch();
        h->sync();
    });
}

sdsl_status sdsl_solve(sdsl_handle h, const double* b, double* x, double tol, int32_t* iters, double* relres) {
    if (!h) return SDSL_E_INVALID;
    sdsl_status result = SDSL_OK;
    sdsl_status st = guard(h, [&] {
        if (!b || !x) fail(SDSL_E_INVALID, "null vector");
        if (!(tol > 0.0)) fail(SDSL_E_INVALID, "tol must be positive");
        SolveTask t;
        t.begin(h, b, x, tol);
        while (!t.finished) t.step();
        if (iters) *iters = t.total_its;
        if (relres) *relres = t.relres;
        result = t.status;
        if (result != SDSL_OK)
            h->err = result == SDSL_E_BREAKDOWN ? "Krylov breakdown" : "tolerance not reached";
    });
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

sdsl_status sdsl_get_info(sdsl_handle h, sdsl_info* out) {
    if (!h || !out) return SDSL_E_INVALID;
    *out = h->info;
    out->device_bytes = (int64_t)h->bytes;
    return SDSL_OK;
}

const char* sdsl_last_error(sdsl_handle h) { return h ? h->err.c_str() : g_thread_err.c_str(); }

void sdsl_destroy(sdsl_handle h) { delete h; }

sdsl_status sdsl_spmv(sdsl_handle h, int32_t prec, const void* x, void* y) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!x || !y) fail(SDSL_E_INVALID, "null vector");
        const CsrView A{h->n, h->rp, h->ci};
        if (prec == SDSL_FP64) {
            if (h->lr64.k > 0) launch_lowrank_tdot<double>(h->lr64, (const double*)x, nullptr, h->s);
            launch_spmv<double>(A, h->v, h->lr64, (const double*)x, (double*)y, nullptr, nullptr, h->lanes, h->grid,
                                h->s);
        } else {
            if (h->lr32.k > 0) launch_lowrank_tdot<float>(h->lr32, (const float*)x, nullptr, h->s);
            launch_spmv<float>(A, h->v32, h->lr32, (const float*)x, (float*)y, nullptr, nullptr, h->lanes, h->grid,
                               h->s);
        }
        h->check_launch();
        h->sync();
    });
}

sdsl_status sdsl_precond_apply(sdsl_handle h, int32_t prec, const void* r, void* z) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!r || !z) fail(SDSL_E_INVALID, "null vector");
        PcgVecs V{};
        V.r = const_cast<void*>(r);
        V.z = z;
        hip_check(hipMemsetAsync(h->spin_err, 0, sizeof(int), h->s), "memset");
        if (prec == SDSL_FP64) {
            V.y = h->y;
            launch_bj<double>(0, bj_dev(h, false), V, nullptr, 0, h->s);
        } else {
            V.y = h->y32;
            launch_bj<float>(0, bj_dev(h, true), V, nullptr, 0, h->s);
        }
        h->check_launch();
        h->sync();
    });
}

sdsl_status sdsl_residual(sdsl_handle h, const double* b, const double* x, double* r, double* norm) {
    if (!h) return SDSL_E_INVALID;
    return guard(h, [&] {
        if (!b || !x || !r) fail(SDSL_E_INVALID, "null vector");
        const double nr = true_residual(h, b, x, r);
        if (norm) *norm = nr;
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

}  // extern "C"
