// Preconditioner construction on gfx950: input validation, the sparse filter
// with diagonal correction, and the batched ILU(0) of all diagonal blocks in
// one launch.
#include <climits>

#include "common.hpp"

namespace sdsl {

// ---------------------------------------------------------------- validation
__global__ void k_validate(int n, const int64_t* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, ValidateOut* out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int64_t a = rp[i], b = rp[i + 1];
        if (b < a) {
            atomicAdd(&out->bad_rowptr, 1);
            atomicMin(&out->first_bad, i);
            continue;
        }
        int prev = -1;
        bool bad = false, diag = false, nonfinite = false;
        for (int64_t p = a; p < b; ++p) {
            const int c = ci[p];
            if (c <= prev || c >= n) bad = true;
            if (c == i) diag = true;
            if (!isfinite(v[p])) nonfinite = true;
            prev = c;
        }
        if (bad) atomicAdd(&out->bad_rows, 1);
        if (!diag) atomicAdd(&out->missing_diag, 1);
        if (nonfinite) atomicAdd(&out->nonfinite, 1);
        if (bad || !diag || nonfinite) atomicMin(&out->first_bad, i);
    }
}

__global__ void k_vout_init(ValidateOut* out) {
    out->bad_rows = 0;
    out->missing_diag = 0;
    out->nonfinite = 0;
    out->bad_rowptr = 0;
    out->first_bad = INT_MAX;
}

void launch_validate(int n, const int64_t* rp64, const int* ci, const double* v, ValidateOut* out,
                     hipStream_t s) {
    k_vout_init<<<1, 1, 0, s>>>(out);
    const int grid = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    if (n > 0) k_validate<<<grid > 0 ? grid : 1, 256, 0, s>>>(n, rp64, ci, v, out);
}

__global__ void k_nonfinite(int64_t m, const double* __restrict__ v, ValidateOut* out) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        bad += !isfinite(v[i]);
    if (bad) atomicAdd(&out->nonfinite, bad);
}
void launch_count_nonfinite(int64_t m, const double* v, ValidateOut* out, hipStream_t s) {
    k_vout_init<<<1, 1, 0, s>>>(out);
    if (m <= 0) return;
    const int64_t g = (m + 255) / 256;
    k_nonfinite<<<(int)(g < 4096 ? g : 4096), 256, 0, s>>>(m, v, out);
}

__global__ void k_rowptr32(int n, const int64_t* __restrict__ a, int* __restrict__ b) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
        b[i] = (int)a[i];
}
void launch_rowptr32(int n, const int64_t* rp64, int* rp32, hipStream_t s) {
    const int grid = (n + 256) / 256 < 4096 ? (n + 256) / 256 : 4096;
    k_rowptr32<<<grid, 256, 0, s>>>(n, rp64, rp32);
}

__global__ void k_cast_f32(int64_t m, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}
void launch_cast_f32(int64_t m, const double* a, float* b, hipStream_t s) {
    if (m <= 0) return;
    int64_t g = (m + 255) / 256;
    k_cast_f32<<<(int)(g < 8192 ? g : 8192), 256, 0, s>>>(m, a, b);
}

__global__ void k_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                       const double* __restrict__ v, double* __restrict__ d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        // binary search for column i in the sorted row
        int lo = rp[i], hi = rp[i + 1];
        double val = 0.0;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int c = ci[mid];
            if (c == i) { val = v[mid]; break; }
            if (c < i) lo = mid + 1; else hi = mid;
        }
        d[i] = val;
    }
}
void launch_diag(int n, const int* rp, const int* ci, const double* v, double* diag, hipStream_t s) {
    const int grid = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    if (n > 0) k_diag<<<grid, 256, 0, s>>>(n, rp, ci, v, diag);
}

// ---------------------------------------------------------------- filter
// Eq. (filter) (MIN) or its unit-diagonal form (GEOMEAN); evaluated exactly as
// written, with no contraction, so that the kept pattern is a function of the
// FP64 values alone.
__device__ __forceinline__ bool dropped(int mode, double a, double dii, double djj, double tau) {
    if (mode == SDSL_FILTER_MIN)
        return (fabs(a) < tau * fabs(dii)) && (fabs(a) < tau * fabs(djj));
    if (mode == SDSL_FILTER_GEOMEAN) {
        const double lhs = a * a;
        const double rhs = (tau * tau) * (fabs(dii) * fabs(djj));
        return lhs < rhs;
    }
    return false;
}

__device__ __forceinline__ int block_of(const int* bp, int nblocks, int i) {
    int lo = 0, hi = nblocks;  // bp[lo] <= i < bp[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bp[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_filter_count(int n_int, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ v, const double* __restrict__ diag,
                               const int* __restrict__ bp, int nblocks, int mode, double tau,
                               int* __restrict__ cnt, double* __restrict__ dropsum) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_int; i += gridDim.x * blockDim.x) {
        const int b = block_of(bp, nblocks, i);
        const int lo = bp[b], hi = bp[b + 1];
        const double dii = diag[i];
        int c = 0;
        double ds = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (j < lo || j >= hi) continue;
            const double a = v[p];
            if (j != i && dropped(mode, a, dii, diag[j], tau)) { ds += fabs(a); continue; }
            ++c;
        }
        cnt[i] = c;
        dropsum[i] = ds;
    }
}
void launch_filter_count(int n_int, const int* rp, const int* ci, const double* v, const double* diag,
                         const int* bp, int nblocks, int mode, double tau, int* cnt, double* dropsum,
                         hipStream_t s) {
    const int grid = (n_int + 255) / 256 < 8192 ? (n_int + 255) / 256 : 8192;
    if (n_int > 0)
        k_filter_count<<<grid, 256, 0, s>>>(n_int, rp, ci, v, diag, bp, nblocks, mode, tau, cnt, dropsum);
}

__global__ void k_filter_compact(int n_int, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const double* __restrict__ v, const double* __restrict__ diag,
                                 const int* __restrict__ bp, int nblocks, int mode, double tau,
                                 unsigned flags, double delta, const double* __restrict__ dropsum,
                                 const int* __restrict__ prp, int* __restrict__ pci,
                                 double* __restrict__ pv, int* __restrict__ pdiag) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_int; i += gridDim.x * blockDim.x) {
        const int b = block_of(bp, nblocks, i);
        const int lo = bp[b], hi = bp[b + 1];
        const double dii = diag[i];
        int w = prp[i], dpos = -1;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int j = ci[p];
            if (j < lo || j >= hi) continue;
            const double a = v[p];
            if (j != i && dropped(mode, a, dii, diag[j], tau)) continue;
            if (j == i) dpos = w;
            pci[w] = j;
            pv[w] = a;
            ++w;
        }
        pdiag[i] = dpos;
        // Eq. (diagcorr): p_ii + sign(p_ii) * (delta [+ dropsum_i]), sign(0) = +1
        if (flags & (SDSL_DIAG_DELTA | SDSL_DIAG_DROPSUM)) {
            double corr = 0.0;
            if (flags & SDSL_DIAG_DELTA) corr = delta;
            if (flags & SDSL_DIAG_DROPSUM) corr = corr + dropsum[i];
            const double d = pv[dpos];
            pv[dpos] = (d >= 0.0) ? d + corr : d - corr;
        }
    }
}
void launch_filter_compact(int n_int, const int* rp, const int* ci, const double* v, const double* diag,
                           const int* bp, int nblocks, int mode, double tau, unsigned flags,
                           double delta, const double* dropsum, const int* prp, int* pci,
                           double* pv_corr, int* pdiag, hipStream_t s) {
    const int grid = (n_int + 255) / 256 < 8192 ? (n_int + 255) / 256 : 8192;
    if (n_int > 0)
        k_filter_compact<<<grid, 256, 0, s>>>(n_int, rp, ci, v, diag, bp, nblocks, mode, tau, flags, delta,
                                              dropsum, prp, pci, pv_corr, pdiag);
}

// ---------------------------------------------------------------- scan
// Exclusive scan of int counts in three passes over 1024-element tiles.
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
    // Hillis-Steele over the 1024 threads in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int add = (t >= o) ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int incl = sh[t];
    *total = sh[1023];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(1024) void k_scan_tiles(int n, const int* __restrict__ cnt, int* __restrict__ tsum) {
    __shared__ int sh[1024];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    int tot;
    block_excl_scan(i < n ? cnt[i] : 0, sh, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int nt, int* __restrict__ tsum) {
    __shared__ int sh[1024];
    int carry = 0;
    for (int base = 0; base < nt; base += 1024) {
        const int i = base + threadIdx.x;
        int tot;
        const int ex = block_excl_scan(i < nt ? tsum[i] : 0, sh, &tot);
        if (i < nt) tsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[nt] = carry;
}

__global__ __launch_bounds__(1024) void k_scan_apply(int n, const int* __restrict__ cnt,
                                                     const int* __restrict__ tsum, int* __restrict__ out,
                                                     int nt) {
    __shared__ int sh[1024];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    int tot;
    const int ex = block_excl_scan(i < n ? cnt[i] : 0, sh, &tot);
    if (i < n) out[i] = tsum[blockIdx.x] + ex;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tsum[nt];
}

void launch_scan(int n, const int* cnt, int* out, int* tmp, hipStream_t s) {
    const int nt = (n + 1023) / 1024;
    if (nt == 0) {
        (void)hipMemsetAsync(out, 0, sizeof(int), s);
        return;
    }
    k_scan_tiles<<<nt, 1024, 0, s>>>(n, cnt, tmp);
    k_scan_top<<<1, 1024, 0, s>>>(nt, tmp);
    k_scan_apply<<<nt, 1024, 0, s>>>(n, cnt, tmp, out, nt);
}

// ---------------------------------------------------------------- ILU(0)
// One workgroup per diagonal block, all blocks in one launch (paper Sec. 2.3:
// the blocks are independent in factorisation).  Rows are taken in chunks of
// blockDim.x consecutive rows, one row per thread.  Inside a chunk a row waits
// for the rows k < i of its pattern through per-row ready flags in LDS
// (release/acquire at workgroup scope); rows of earlier chunks are complete
// after the chunk barrier.  No lane ever blocks inside a wait: every pass of
// the outer loop lets each lane advance as far as its dependencies allow, so
// the smallest unfinished row always progresses and lanes of one wavefront
// cannot starve each other.  The wait is bounded; running out sets spin_err
// and the kernel still terminates.
//
// Per row i (IKJ ILU(0)): for k in pattern(i), k < i, ascending:
//   l_ik = p_ik / u_kk;  p_ij = fma(-l_ik, u_kj, p_ij) for j > k in both rows.
constexpr int kIluThreads = 1024;
constexpr int kSpinLimit = 1 << 24;

__global__ __launch_bounds__(kIluThreads) void k_ilu0(const int* __restrict__ bp, const int* __restrict__ prp,
                                                      const int* __restrict__ pci,
                                                      const double* __restrict__ pv_corr,
                                                      double* __restrict__ pv, const int* __restrict__ pdiag,
                                                      int spd, int policy, double shift0,
                                                      double* __restrict__ shifts, int* __restrict__ nfix,
                                                      int* __restrict__ block_status, int* spin_err) {
    __shared__ int ready[kIluThreads];
    __shared__ int failed;
    __shared__ int fixes;
    const int b = blockIdx.x, t = threadIdx.x;
    const int lo = bp[b], hi = bp[b + 1];
    double a = 0.0;
    int status = 0;
    for (int attempt = 0;; ++attempt) {
        // working copy of the corrected block, diagonals raised by the shift
        for (int e = prp[lo] + t; e < prp[hi]; e += kIluThreads) pv[e] = pv_corr[e];
        __syncthreads();
        if (a != 0.0)
            for (int i = lo + t; i < hi; i += kIluThreads) {
                const double d = pv_corr[pdiag[i]];
                pv[pdiag[i]] = d + a * d;
            }
        if (t == 0) { failed = 0; fixes = 0; }
        __syncthreads();
        for (int c0 = lo; c0 < hi; c0 += kIluThreads) {
            ready[t] = 0;
            __syncthreads();
            const int i = c0 + t;
            bool fin = (i >= hi);
            int p = fin ? 0 : prp[i];
            const int pd = fin ? 0 : pdiag[i];
            const int pe = fin ? 0 : prp[i + 1];
            const double orig = fin ? 0.0 : pv[pd];
            int spins = 0;
            while (true) {
                if (!fin) {
                    while (p < pd) {
                        const int k = pci[p];
                        if (k >= c0 &&
                            __hip_atomic_load(&ready[k - c0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
                            break;
                        const int kd = pdiag[k];
                        const double l = pv[p] / pv[kd];
                        pv[p] = l;
                        int q = kd + 1, s = p + 1;
                        const int qe = prp[k + 1];
                        while (q < qe && s < pe) {
                            const int cq = pci[q], cs = pci[s];
                            if (cq < cs) ++q;
                            else if (cq > cs) ++s;
                            else { pv[s] = fma(-l, pv[q], pv[s]); ++q; ++s; }
                        }
                        ++p;
                    }
                    if (p == pd) {
                        const double u = pv[pd];
                        const bool bad = spd ? !(u > 0.0) : !(fabs(u) >= 1e-14 * fabs(orig));
                        if (bad) {
                            if (policy == SDSL_PIVOT_REPLACE) {
                                pv[pd] = orig;
                                atomicAdd(&fixes, 1);
                            } else {
                                failed = 1;
                            }
                        }
                        __hip_atomic_store(&ready[t], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        fin = true;
                    }
                }
                if (__all(fin)) break;
                if (++spins > kSpinLimit) {
                    if (!fin) {
                        atomicExch(spin_err, 1);
                        failed = 1;
                        __hip_atomic_store(&ready[t], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        fin = true;
                    }
                }
            }
            __syncthreads();
            if (failed) break;
        }
        __syncthreads();
        const int f = failed;
        __syncthreads();
        if (!f) break;
        if (policy != SDSL_PIVOT_SHIFT || attempt >= 48) { status = SDSL_E_BREAKDOWN; break; }
        a = (a == 0.0) ? shift0 : 2.0 * a;
        __syncthreads();
    }
    if (t == 0) {
        shifts[b] = status ? -1.0 : a;
        block_status[b] = status;
        if (fixes) atomicAdd(nfix, fixes);
    }
}

__global__ void k_lu_counts(int n, const int* __restrict__ prp, const int* __restrict__ pdiag, int* __restrict__ lc,
                            int* __restrict__ uc) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        lc[i] = pdiag[i] - prp[i];
        uc[i] = prp[i + 1] - pdiag[i] - 1;
    }
}
void launch_lu_counts(int n_int, const int* prp, const int* pdiag, int* lcnt, int* ucnt, hipStream_t s) {
    const int g = (n_int + 255) / 256 < 4096 ? (n_int + 255) / 256 : 4096;
    if (n_int > 0) k_lu_counts<<<g, 256, 0, s>>>(n_int, prp, pdiag, lcnt, ucnt);
}
__global__ void k_lu_split(int n, const int* __restrict__ prp, const int* __restrict__ pci,
                           const double* __restrict__ pv, const int* __restrict__ pdiag, const int* __restrict__ lrp,
                           int* __restrict__ lci, double* __restrict__ lval, const int* __restrict__ urp,
                           int* __restrict__ uci, double* __restrict__ uval, double* __restrict__ udiag) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int a = prp[i], d = pdiag[i], e = prp[i + 1];
        int w = lrp[i];
        for (int p = a; p < d; ++p, ++w) { lci[w] = pci[p]; lval[w] = pv[p]; }
        // U rows in descending column order: the backward substitution
        // takes its terms in the order their unknowns are solved
        w = urp[i];
        for (int p = e - 1; p > d; --p, ++w) { uci[w] = pci[p]; uval[w] = pv[p]; }
        udiag[i] = pv[d];
    }
}
void launch_lu_split(int n_int, const int* prp, const int* pci, const double* pv, const int* pdiag, const int* lrp,
                     int* lci, double* lval, const int* urp, int* uci, double* uval, double* udiag, hipStream_t s) {
    const int g = (n_int + 255) / 256 < 4096 ? (n_int + 255) / 256 : 4096;
    if (n_int > 0) k_lu_split<<<g, 256, 0, s>>>(n_int, prp, pci, pv, pdiag, lrp, lci, lval, urp, uci, uval, udiag);
}

void launch_ilu0(int nblocks, const int* bp, const int* prp, const int* pci, const double* pv_corr,
                 double* pv, const int* pdiag, int spd, int policy, double shift0, double* shifts,
                 int* nfix, int* block_status, int* spin_err, hipStream_t s) {
    if (nblocks <= 0) return;
    k_ilu0<<<nblocks, kIluThreads, 0, s>>>(bp, prp, pci, pv_corr, pv, pdiag, spd, policy, shift0, shifts, nfix,
                                          block_status, spin_err);
}

}  // namespace sdsl
