// Per-iteration kernels on gfx950: CSR SpMV with fused dot, compensated FP64
// residual, the block-Jacobi apply (forward + backward substitution of every
// block in one launch, fused with the PCG vector updates) and the PCG
// direction update.
#include "common.hpp"

namespace sdsl {

constexpr int kSpinLimitIter = 1 << 24;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ bool krylov_done(const KrylovState* st) {
    return __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Block-uniform read of the done flag (one read, broadcast through LDS).
__device__ __forceinline__ bool block_done(const KrylovState* st, int* sh) {
    if (threadIdx.x == 0) *sh = st ? (krylov_done(st) ? 1 : 0) : 0;
    __syncthreads();
    const bool d = *sh != 0;
    __syncthreads();
    return d;
}

__device__ __forceinline__ void set_done(KrylovState* st) {
    __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Logical workgroup index with consecutive row ranges kept on one XCD: the
// hardware deals workgroups round-robin over the 8 XCDs, so workgroup w runs
// on XCD w % 8; mapping it to range (w % 8) * (G / 8) + w / 8 gives every XCD
// one contiguous eighth of the rows (and of the x entries they gather).
__device__ __forceinline__ int xcd_swizzle(int w, int g) {
    return (g % 8 == 0) ? (w % 8) * (g / 8) + (w / 8) : w;
}

int spmv_grid(int n) {
    // 8 workgroups of 256 threads per CU over 256 CUs at most; a multiple of 8
    int g = (n + 63) / 64;
    if (g > 2048) g = 2048;
    g = (g + 7) / 8 * 8;
    return g < 8 ? 8 : g;
}

int spmv_lanes(double mean_row) {
    if (mean_row >= 96) return 64;
    if (mean_row >= 40) return 32;
    if (mean_row >= 20) return 16;
    if (mean_row >= 8) return 8;
    return 4;
}

// ------------------------------------------------------------------ low rank
// part[j * slices + s] = sum over slice s of column j of U^T x (FP64).  With
// COMP the slice sums are compensated and their error terms go to
// part[k * slices + j * slices + s].
template <typename T, bool COMP>
__global__ __launch_bounds__(256) void k_lowrank_tdot(int k, int slices, const int* __restrict__ ucp,
                                                      const int* __restrict__ uri, const T* __restrict__ ucv,
                                                      const T* __restrict__ x, double* __restrict__ part,
                                                      const KrylovState* st) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const int j = blockIdx.x / slices, s = blockIdx.x % slices;
    const int a = ucp[j], e = ucp[j + 1];
    const int len = e - a;
    const int lo = a + (int)((int64_t)len * s / slices), hi = a + (int)((int64_t)len * (s + 1) / slices);
    double sum = 0.0, err = 0.0;
    for (int p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        const double pr = (double)ucv[p] * (double)x[uri[p]];
        if (COMP) {
            const double pe = fma((double)ucv[p], (double)x[uri[p]], -pr);
            const double t = sum + pr;
            const double z = t - sum;
            err += (sum - (t - z)) + (pr - z) + pe;
            sum = t;
        } else {
            sum += pr;
        }
    }
    if (COMP) {
        // fold the per-thread pairs; the error terms are summed separately
        const double tot = block_sum(sum, red);
        // error of combining the thread sums is bounded by u*sum(|sum_t|); add
        // the per-thread corrections, which dominate for long columns
        const double terr = block_sum(err, red);
        if (threadIdx.x == 0) {
            part[j * slices + s] = tot;
            part[k * slices + j * slices + s] = terr;
        }
    } else {
        const double tot = block_sum(sum, red);
        if (threadIdx.x == 0) part[j * slices + s] = tot;
    }
}

template <typename T>
void launch_lowrank_tdot(const LowRankDev& lr, const T* x, const KrylovState* st, hipStream_t s) {
    if (lr.k <= 0) return;
    k_lowrank_tdot<T, false><<<lr.k * lr.slices, 256, 0, s>>>(lr.k, lr.slices, lr.ucp, lr.uri,
                                                              (const T*)lr.ucv, x, lr.part, st);
}
template void launch_lowrank_tdot<double>(const LowRankDev&, const double*, const KrylovState*, hipStream_t);
template void launch_lowrank_tdot<float>(const LowRankDev&, const float*, const KrylovState*, hipStream_t);

// ------------------------------------------------------------------ SpMV
// y = M x (+ U diag(c) U^T x) with G lanes per row.  Values and column
// indices are streamed with non-temporal loads so that the gathered x stays
// in L2; each workgroup owns one contiguous row range (XCD-swizzled).  With
// part_dot the workgroup's share of (x, y) is written to part_dot[w].
template <typename T, int G, bool LR>
__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const T* __restrict__ v, const T* __restrict__ x,
                                              T* __restrict__ y, double* __restrict__ part_dot,
                                              const KrylovState* st, LowRankDev lr) {
    __shared__ double red[8];
    __shared__ T tk[64];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    if (LR) {
        const T* c = (const T*)lr.c;
        for (int j = threadIdx.x; j < lr.k; j += blockDim.x) {
            double s = 0.0;
            for (int q = 0; q < lr.slices; ++q) s += lr.part[j * lr.slices + q];
            tk[j] = (T)((double)c[j] * s);
        }
        __syncthreads();
    }
    const int g = gridDim.x;
    const int lw = xcd_swizzle(blockIdx.x, g);
    const int per = (n + g - 1) / g;
    const int r0 = lw * per;
    const int r1 = min(n, r0 + per);
    constexpr int RPW = 256 / G;  // rows in flight per workgroup
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    double dacc = 0.0;
    for (int row = r0 + grp; row < r1; row += RPW) {
        const int a = rp[row], e = rp[row + 1];
        T s0 = T(0), s1 = T(0);
        int p = a + lane;
        for (; p + G < e; p += 2 * G) {
            const T v0 = __builtin_nontemporal_load(&v[p]);
            const int c0 = __builtin_nontemporal_load(&ci[p]);
            const T v1 = __builtin_nontemporal_load(&v[p + G]);
            const int c1 = __builtin_nontemporal_load(&ci[p + G]);
            s0 = fma(v0, x[c0], s0);
            s1 = fma(v1, x[c1], s1);
        }
        if (p < e) s0 = fma(__builtin_nontemporal_load(&v[p]), x[__builtin_nontemporal_load(&ci[p])], s0);
        T s = group_sum<G>(s0 + s1);
        if (lane == 0) {
            if (LR) {
                const T* uv = (const T*)lr.uv;
                for (int q = lr.urp[row]; q < lr.urp[row + 1]; ++q) s = fma(uv[q], tk[lr.uci[q]], s);
            }
            y[row] = s;
            if (part_dot) dacc += (double)x[row] * (double)s;
        }
    }
    if (part_dot) {
        const double tot = block_sum(dacc, red);
        if (threadIdx.x == 0) part_dot[blockIdx.x] = tot;
    }
}

template <typename T, bool LR>
static void spmv_dispatch(const CsrView& A, const T* v, const LowRankDev& lr, const T* x, T* y, double* pd,
                          const KrylovState* st, int lanes, int grid, hipStream_t s) {
    switch (lanes) {
        case 64: k_spmv<T, 64, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        case 32: k_spmv<T, 32, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        case 16: k_spmv<T, 16, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        case 8: k_spmv<T, 8, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        default: k_spmv<T, 4, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
    }
}

template <typename T>
void launch_spmv(const CsrView& A, const T* v, const LowRankDev& lr, const T* x, T* y, double* part_dot,
                 const KrylovState* st, int lanes, int grid, hipStream_t s) {
    if (lr.k > 0) spmv_dispatch<T, true>(A, v, lr, x, y, part_dot, st, lanes, grid, s);
    else spmv_dispatch<T, false>(A, v, lr, x, y, part_dot, st, lanes, grid, s);
}
template void launch_spmv<double>(const CsrView&, const double*, const LowRankDev&, const double*, double*,
                                  double*, const KrylovState*, int, int, hipStream_t);
template void launch_spmv<float>(const CsrView&, const float*, const LowRankDev&, const float*, float*,
                                 double*, const KrylovState*, int, int, hipStream_t);

// ------------------------------------------------------------------ residual
// r = b - M x (- U diag(c) U^T x) with every row accumulated as an
// error-free (TwoProduct / TwoSum) pair, then rounded once; part[w] gets the
// workgroup's share of ||r||^2.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

template <int G, bool LR>
__global__ __launch_bounds__(256) void k_residual(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double* __restrict__ v, const double* __restrict__ b,
                                                  const double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ part, LowRankDev lr) {
    __shared__ double red[8];
    __shared__ double tk[64];
    if (LR) {
        const double* c = (const double*)lr.c;
        for (int j = threadIdx.x; j < lr.k; j += blockDim.x) {
            double s = 0.0, e = 0.0;
            for (int q = 0; q < lr.slices; ++q) {
                double t, te;
                two_sum(s, lr.part[j * lr.slices + q], t, te);
                s = t;
                e += te + lr.part[lr.k * lr.slices + j * lr.slices + q];
            }
            tk[j] = c[j] * (s + e);
        }
        __syncthreads();
    }
    const int g = gridDim.x;
    const int lw = xcd_swizzle(blockIdx.x, g);
    const int per = (n + g - 1) / g;
    const int r0 = lw * per, r1 = min(n, r0 + per);
    constexpr int RPW = 256 / G;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    double sq = 0.0;
    for (int row = r0 + grp; row < r1; row += RPW) {
        double s = (lane == 0) ? b[row] : 0.0, e = 0.0;
        for (int p = rp[row] + lane; p < rp[row + 1]; p += G) {
            const double pr = -v[p] * x[ci[p]];
            const double pe = fma(-v[p], x[ci[p]], -pr);
            double t, te;
            two_sum(s, pr, t, te);
            s = t;
            e += pe + te;
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            const double so = __shfl_xor(s, o, kWave), eo = __shfl_xor(e, o, kWave);
            double t, te;
            two_sum(s, so, t, te);
            s = t;
            e = e + eo + te;
        }
        if (lane == 0) {
            if (LR) {
                const double* uv = (const double*)lr.uv;
                for (int q = lr.urp[row]; q < lr.urp[row + 1]; ++q) {
                    const double pr = -uv[q] * tk[lr.uci[q]];
                    const double pe = fma(-uv[q], tk[lr.uci[q]], -pr);
                    double t, te;
                    two_sum(s, pr, t, te);
                    s = t;
                    e += pe + te;
                }
            }
            const double ri = s + e;
            r[row] = ri;
            sq += ri * ri;
        }
    }
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

void launch_residual(const CsrView& A, const double* v, const LowRankDev& lr, const double* b,
                     const double* x, double* r, double* part, int lanes, int grid, hipStream_t s) {
    if (lr.k > 0)
        k_lowrank_tdot<double, true><<<lr.k * lr.slices, 256, 0, s>>>(lr.k, lr.slices, lr.ucp, lr.uri,
                                                                      (const double*)lr.ucv, x, lr.part,
                                                                      nullptr);
#define RES_CASE(G)                                                                                  \
    case G:                                                                                          \
        if (lr.k > 0) k_residual<G, true><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, b, x, r, part, lr); \
        else k_residual<G, false><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, b, x, r, part, lr);        \
        break;
    switch (lanes) {
        RES_CASE(64)
        RES_CASE(32)
        RES_CASE(16)
        RES_CASE(8)
        default:
        RES_CASE(4)
    }
#undef RES_CASE
}

// ------------------------------------------------------------------ reductions
__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ part, int m, double* out) {
    __shared__ double red[16];
    const double s = block_sum_array(part, m, red);
    if (threadIdx.x == 0) out[0] = s;
}
void launch_sum_partials(const double* part, int m, double* out, hipStream_t s) {
    k_sum_partials<<<1, 1024, 0, s>>>(part, m, out);
}

__global__ __launch_bounds__(256) void k_sqnorm_partials(int n, const double* __restrict__ a,
                                                         double* __restrict__ part) {
    __shared__ double red[8];
    const int g = gridDim.x;
    const int per = (n + g - 1) / g;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double s = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) s += a[i] * a[i];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}
void launch_sqnorm_partials(int n, const double* a, double* part, int grid, hipStream_t s) {
    k_sqnorm_partials<<<grid, 256, 0, s>>>(n, a, part);
}

// st <- fresh state with bb = sum(part[0..m)) and tol2 = tol^2
__global__ __launch_bounds__(1024) void k_init_state(KrylovState* st, const double* part, int m, double tol) {
    __shared__ double red[16];
    const double s = block_sum_array(part, m, red);
    if (threadIdx.x == 0) {
        st->conv = 0;
        st->breakdown = 0;
        st->iters = 0;
        st->spin_err = 0;
        st->bb = s;
        st->tol2 = tol * tol;
        __hip_atomic_store(&st->done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
void launch_init_state(KrylovState* st, const double* part_bb, int m, double tol, hipStream_t s) {
    k_init_state<<<1, 1024, 0, s>>>(st, part_bb, m, tol);
}

// ------------------------------------------------------------------ vectors
template <typename T>
__global__ void k_fill(int64_t n, T* a, T val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = val;
}
template <typename T>
void launch_fill(int64_t n, T* a, T val, hipStream_t s) {
    if (n <= 0) return;
    const int64_t g = (n + 255) / 256;
    k_fill<T><<<(int)(g < 4096 ? g : 4096), 256, 0, s>>>(n, a, val);
}
template void launch_fill<double>(int64_t, double*, double, hipStream_t);
template void launch_fill<float>(int64_t, float*, float, hipStream_t);
template void launch_fill<int>(int64_t, int*, int, hipStream_t);

template <typename T>
__global__ void k_copy(int64_t n, const T* __restrict__ a, T* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}
template <typename T>
void launch_copy(int64_t n, const T* a, T* b, hipStream_t s) {
    if (n <= 0) return;
    const int64_t g = (n + 255) / 256;
    k_copy<T><<<(int)(g < 4096 ? g : 4096), 256, 0, s>>>(n, a, b);
}
template void launch_copy<double>(int64_t, const double*, double*, hipStream_t);
template void launch_copy<float>(int64_t, const float*, float*, hipStream_t);

// rs = fl32(r / nr), nr = sqrt(*nr2)
__global__ void k_ir_scale_cast(int n, const double* __restrict__ r, const double* __restrict__ nr2,
                                float* __restrict__ rs) {
    const double nr = sqrt(nr2[0]);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        rs[i] = (float)(r[i] / nr);
}
void launch_ir_scale_cast(int n, const double* r, const double* nr2, float* rs, hipStream_t s) {
    const int g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    k_ir_scale_cast<<<g > 0 ? g : 1, 256, 0, s>>>(n, r, nr2, rs);
}

// x += nr * d in FP64
__global__ void k_ir_update(int n, double* __restrict__ x, const double* __restrict__ nr2,
                            const float* __restrict__ d) {
    const double nr = sqrt(nr2[0]);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] = x[i] + nr * (double)d[i];
}
void launch_ir_update(int n, double* x, const double* nr2, const float* d, hipStream_t s) {
    const int g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    k_ir_update<<<g > 0 ? g : 1, 256, 0, s>>>(n, x, nr2, d);
}

// ------------------------------------------------------------------ BJ apply
// One workgroup per diagonal block (all blocks in one launch).  Forward
// substitution y = L^{-1} r then backward substitution z = U^{-1} y, each
// over chunks of 1024 consecutive rows with one row per thread.  The block's
// most recent kRing solution values live in an LDS ring (slot = local row mod
// kRing); a slot of the current chunk holds the sentinel until its row is
// final, so a row waits on a same-chunk dependency by re-reading the slot.
// Dependencies in earlier chunks are final after the chunk barrier and are
// read from the ring, or from global memory once evicted.  Each row sums its
// terms in pattern order, so the result is a fixed function of the inputs.
constexpr int kBjThreads = 1024;
constexpr int kRing = 8192;

template <typename T>
__device__ __forceinline__ T from_bits(typename Sentinel<T>::Bits b) {
    T v;
    __builtin_memcpy(&v, &b, sizeof(T));
    return v;
}
template <typename T>
__device__ __forceinline__ typename Sentinel<T>::Bits to_bits(T v) {
    typename Sentinel<T>::Bits b;
    __builtin_memcpy(&b, &v, sizeof(T));
    return b;
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBjThreads) void k_bj(BJDev P, PcgVecs V, KrylovState* st, int it) {
    using Bits = typename Sentinel<T>::Bits;
    constexpr Bits SENT = Sentinel<T>::bits;
    __shared__ Bits ring[kRing];
    __shared__ double red[16];
    __shared__ int shd;
    const int b = blockIdx.x, t = threadIdx.x;
    const int nb = P.nblocks;
    const int lo = P.bp[b], hi = P.bp[b + 1];
    const T* __restrict__ pv = (const T*)P.pv;
    const int* __restrict__ prp = P.prp;
    const int* __restrict__ pci = P.pci;
    const int* __restrict__ pdiag = P.pdiag;
    T* __restrict__ z = (T*)V.z;
    T* __restrict__ y = (T*)V.y;
    T* r = (T*)V.r;

    if (MODE == 1) {
        if (block_done(st, &shd)) return;
        const double pq = block_sum_array(V.part_pq, V.npq, red);
        const double rz_old = block_sum_array(V.part_rz + ((it + 1) & 1) * nb, nb, red);
        const double alpha = rz_old / pq;
        if (!(pq > 0.0) || !isfinite(alpha)) {
            if (b == 0 && t == 0) {
                st->breakdown = 1;
                st->iters = it;
                set_done(st);
            }
            return;
        }
        const T a = (T)alpha;
        T* x = (T*)V.x;
        const T* p = (const T*)V.p;
        const T* q = (const T*)V.q;
        double rr = 0.0;
        for (int i = lo + t; i < hi; i += kBjThreads) {
            x[i] = x[i] + a * p[i];
            const T ri = r[i] - a * q[i];
            r[i] = ri;
            rr += (double)ri * (double)ri;
        }
        rr = block_sum(rr, red);
        if (t == 0) V.part_rr[b] = rr;
    }
    const T* rin = r;

    int spin_fail = 0;
    // forward substitution: y_i = r_i - sum_{j<i} l_ij y_j
    for (int c0 = lo; c0 < hi; c0 += kBjThreads) {
        const int i = c0 + t;
        if (i < hi) ring[(i - lo) & (kRing - 1)] = SENT;
        __syncthreads();
        bool fin = i >= hi;
        int pp = fin ? 0 : prp[i];
        const int pe = fin ? 0 : pdiag[i];
        T acc = fin ? T(0) : rin[i];
        const int ring_lo = c0 + kBjThreads - kRing;
        int spins = 0;
        while (true) {
            if (!fin) {
                while (pp < pe) {
                    const int j = pci[pp];
                    T yj;
                    if (j >= c0) {
                        const Bits raw = __hip_atomic_load(&ring[(j - lo) & (kRing - 1)], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (raw == SENT) break;
                        yj = from_bits<T>(raw);
                    } else if (j >= ring_lo) {
                        yj = from_bits<T>(ring[(j - lo) & (kRing - 1)]);
                    } else {
                        yj = y[j];
                    }
                    acc = acc - pv[pp] * yj;
                    ++pp;
                }
                if (pp == pe) {
                    y[i] = acc;
                    __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<T>(acc), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    fin = true;
                }
            }
            if (__all(fin)) break;
            if (++spins > kSpinLimitIter && !fin) {
                spin_fail = 1;
                y[i] = acc;
                __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<T>(acc), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                fin = true;
            }
        }
        __syncthreads();
    }
    // backward substitution: z_i = (y_i - sum_{j>i} u_ij z_j) / u_ii
    for (int c_hi = hi; c_hi > lo; c_hi -= kBjThreads) {
        const int c_lo = max(lo, c_hi - kBjThreads);
        const int i = c_hi - 1 - t;
        if (i >= c_lo) ring[(i - lo) & (kRing - 1)] = SENT;
        __syncthreads();
        bool fin = i < c_lo;
        int pp = fin ? 0 : pdiag[i] + 1;
        const int pe = fin ? 0 : prp[i + 1];
        T acc = fin ? T(0) : y[i];
        const int ring_hi = c_lo + kRing;
        int spins = 0;
        while (true) {
            if (!fin) {
                while (pp < pe) {
                    const int j = pci[pp];
                    T zj;
                    if (j < c_hi) {
                        const Bits raw = __hip_atomic_load(&ring[(j - lo) & (kRing - 1)], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (raw == SENT) break;
                        zj = from_bits<T>(raw);
                    } else if (j < ring_hi) {
                        zj = from_bits<T>(ring[(j - lo) & (kRing - 1)]);
                    } else {
                        zj = z[j];
                    }
                    acc = acc - pv[pp] * zj;
                    ++pp;
                }
                if (pp == pe) {
                    const T zi = acc / pv[pdiag[i]];
                    z[i] = zi;
                    __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<T>(zi), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    fin = true;
                }
            }
            if (__all(fin)) break;
            if (++spins > kSpinLimitIter && !fin) {
                spin_fail = 1;
                z[i] = acc;
                __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<T>(acc), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                fin = true;
            }
        }
        __syncthreads();
    }
    if (spin_fail && st) atomicExch(&st->spin_err, 1);
    if (MODE != 0) {
        double rz = 0.0;
        for (int i = lo + t; i < hi; i += kBjThreads) rz += (double)rin[i] * (double)z[i];
        rz = block_sum(rz, red);
        if (t == 0) V.part_rz[(it & 1) * nb + b] = rz;
    }
}

template <typename T>
void launch_bj(int mode, const BJDev& P, const PcgVecs& v, KrylovState* st, int it, hipStream_t s) {
    if (P.nblocks <= 0) return;
    if (mode == 0) k_bj<T, 0><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it);
    else if (mode == 1) k_bj<T, 1><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it);
    else k_bj<T, 2><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it);
}
template void launch_bj<double>(int, const BJDev&, const PcgVecs&, KrylovState*, int, hipStream_t);
template void launch_bj<float>(int, const BJDev&, const PcgVecs&, KrylovState*, int, hipStream_t);

// ------------------------------------------------------------------ PCG p update
// Convergence test on sum(part_rr) against tol^2 ||b||^2, then
// beta = (r,z)_new / (r,z)_old and p = z + beta p.
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_pupdate(int n, T* __restrict__ p, const T* __restrict__ z,
                                                     const double* __restrict__ part_rz,
                                                     const double* __restrict__ part_rr, int nb,
                                                     KrylovState* st, int it) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const double rr = block_sum_array(part_rr, nb, red);
    if (rr <= st->tol2 * st->bb) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->conv = 1;
            st->iters = it + 1;
            set_done(st);
        }
        return;
    }
    const double rz_new = block_sum_array(part_rz + (it & 1) * nb, nb, red);
    const double rz_old = block_sum_array(part_rz + ((it + 1) & 1) * nb, nb, red);
    const double beta = rz_new / rz_old;
    if (!isfinite(beta)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->breakdown = 1;
            st->iters = it + 1;
            set_done(st);
        }
        return;
    }
    const T bt = (T)beta;
    const int g = gridDim.x;
    const int per = (n + g - 1) / g;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) p[i] = z[i] + bt * p[i];
}

template <typename T>
void launch_pcg_pupdate(int n, const PcgVecs& v, int nblocks, KrylovState* st, int it, hipStream_t s) {
    int g = (n + 1023) / 1024;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    k_pcg_pupdate<T><<<g, 256, 0, s>>>(n, (T*)v.p, (const T*)v.z, v.part_rz, v.part_rr, nblocks, st, it);
}
template void launch_pcg_pupdate<double>(int, const PcgVecs&, int, KrylovState*, int, hipStream_t);
template void launch_pcg_pupdate<float>(int, const PcgVecs&, int, KrylovState*, int, hipStream_t);

}  // namespace sdsl
