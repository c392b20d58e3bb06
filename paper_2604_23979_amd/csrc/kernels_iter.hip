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

// lanes per row of the SpMV: enough that a typical row needs one round of
// U loads per lane (U = 12 for 16 lanes, 8 otherwise)
int spmv_lanes(double mean_row) {
    if (mean_row >= 96) return 16;
    if (mean_row >= 40) return 8;
    if (mean_row >= 16) return 4;
    return 2;
}

// ------------------------------------------------------------------ low rank
// part[j * slices + s] = sum over slice s of column j of U^T x (FP64).  With
// COMP the slice sums are compensated and their error terms go to
// part[k * slices + j * slices + s].
template <typename T, bool COMP>
__global__ __launch_bounds__(256) void k_lowrank_tdot(int k, int slices, const int* __restrict__ ucp,
                                                      const int* __restrict__ uri, const double* __restrict__ ucv,
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
                                                              (const double*)lr.ucv, x, lr.part, st);
}
template void launch_lowrank_tdot<double>(const LowRankDev&, const double*, const KrylovState*, hipStream_t);
template void launch_lowrank_tdot<float>(const LowRankDev&, const float*, const KrylovState*, hipStream_t);

// ------------------------------------------------------------------ SpMV
// y = M x (+ U diag(c) U^T x) with G lanes per row.  Values (type F) and
// column indices are streamed with non-temporal loads so that the gathered x
// (type V) stays in L2; the products and their sum are formed in F (FP32
// values give an FP32 product, accumulated in FP32); the low-rank term is
// added in FP64.  Each workgroup owns one contiguous row range
// (XCD-swizzled).  With part_dot the workgroup's share of (x, y) is written
// to part_dot[w].
template <typename V, typename F, int G, int U, bool LR>
__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const F* __restrict__ v, const V* __restrict__ x,
                                              V* __restrict__ y, double* __restrict__ part_dot,
                                              const KrylovState* st, LowRankDev lr) {
    // Each wave works on batches of 64 consecutive rows: the batch's row
    // bounds are loaded once (coalesced) and broadcast, 64/G rows are in
    // flight per step with G lanes each and U independent loads per lane per
    // round trip (G*U entries per row per round), and the 64 results stay in
    // their lanes until one coalesced store per batch.
    __shared__ double red[8];
    __shared__ double tk[64];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    if (LR) {
        const double* c = (const double*)lr.c;
        for (int j = threadIdx.x; j < lr.k; j += blockDim.x) {
            double s = 0.0;
            for (int q = 0; q < lr.slices; ++q) s += lr.part[j * lr.slices + q];
            tk[j] = c[j] * s;
        }
        __syncthreads();
    }
    constexpr int RPS = kWave / G;  // rows per step per wave
    const int g = gridDim.x;
    const int lw = xcd_swizzle(blockIdx.x, g);
    const int per = (n + g - 1) / g;
    const int r0 = lw * per;
    const int r1 = min(n, r0 + per);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nwaves = blockDim.x / kWave;
    const int grp = lane / G, gl = lane % G;
    double dacc = 0.0;
    for (int base = r0 + wave * kWave; base < r1; base += nwaves * kWave) {
        const int nrow = min(kWave, r1 - base);
        const int my_a = (lane < nrow) ? rp[base + lane] : 0;
        const int my_e = (lane < nrow) ? rp[base + lane + 1] : 0;
        F res = F(0);
#pragma unroll 1
        for (int j = 0; j < kWave; j += RPS) {
            if (j >= nrow) break;
            const int a = __shfl(my_a, j + grp, kWave);
            const int e = __shfl(my_e, j + grp, kWave);
            F s = F(0);
            for (int p0 = a + gl; p0 < e; p0 += U * G) {
                F vv[U];
                int cc[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int p = p0 + u * G;
                    vv[u] = p < e ? __builtin_nontemporal_load(&v[p]) : F(0);
                    cc[u] = p < e ? __builtin_nontemporal_load(&ci[p]) : 0;
                }
                F xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) xv[u] = (p0 + u * G < e) ? (F)x[cc[u]] : F(0);
#pragma unroll
                for (int u = 0; u < U; ++u) s = fma(vv[u], xv[u], s);
            }
            s = group_sum<G>(s);
            // lane L of this step's rows takes the sum of group L - j
            const F mine = __shfl(s, (lane - j) * G, kWave);
            if (lane >= j && lane < j + RPS) res = mine;
        }
        if (lane < nrow) {
            const int row = base + lane;
            V out = (V)res;
            if (LR) {
                const double* uv = (const double*)lr.uv;
                double t = (double)res;
                for (int q = lr.urp[row]; q < lr.urp[row + 1]; ++q) t = fma(uv[q], tk[lr.uci[q]], t);
                out = (V)t;
            }
            y[row] = out;
            if (part_dot) dacc += (double)x[row] * (double)out;
        }
    }
    if (part_dot) {
        const double tot = block_sum(dacc, red);
        if (threadIdx.x == 0) part_dot[blockIdx.x] = tot;
    }
}

template <typename V, typename F, bool LR>
static void spmv_dispatch(const CsrView& A, const F* v, const LowRankDev& lr, const V* x, V* y, double* pd,
                          const KrylovState* st, int lanes, int grid, hipStream_t s) {
    switch (lanes) {
        case 16: k_spmv<V, F, 16, 12, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        case 8: k_spmv<V, F, 8, 8, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        case 4: k_spmv<V, F, 4, 8, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
        default: k_spmv<V, F, 2, 8, LR><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr); break;
    }
}

template <typename V, typename F>
void launch_spmv(const CsrView& A, const F* v, const LowRankDev& lr, const V* x, V* y, double* part_dot,
                 const KrylovState* st, int lanes, int grid, hipStream_t s) {
    if (lr.k > 0) spmv_dispatch<V, F, true>(A, v, lr, x, y, part_dot, st, lanes, grid, s);
    else spmv_dispatch<V, F, false>(A, v, lr, x, y, part_dot, st, lanes, grid, s);
}
template void launch_spmv<double, double>(const CsrView&, const double*, const LowRankDev&, const double*, double*,
                                          double*, const KrylovState*, int, int, hipStream_t);
template void launch_spmv<double, float>(const CsrView&, const float*, const LowRankDev&, const double*, double*,
                                         double*, const KrylovState*, int, int, hipStream_t);
template void launch_spmv<float, float>(const CsrView&, const float*, const LowRankDev&, const float*, float*,
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
__global__ __launch_bounds__(1024) void k_init_state(KrylovState* st, const double* part, int m, double tol,
                                                     double delta) {
    __shared__ double red[16];
    const double s = block_sum_array(part, m, red);
    if (threadIdx.x == 0) {
        st->conv = 0;
        st->breakdown = 0;
        st->iters = 0;
        st->spin_err = 0;
        st->update = 0;
        st->it_refine = 0;
        st->refine_every = 0;
        st->bb = s;
        st->rr0 = s;
        st->tol2 = tol * tol;
        st->delta2 = delta * delta;
        __hip_atomic_store(&st->done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
void launch_init_state(KrylovState* st, const double* part_bb, int m, double tol, double delta, hipStream_t s) {
    k_init_state<<<1, 1024, 0, s>>>(st, part_bb, m, tol, delta);
}

__global__ __launch_bounds__(1024) void k_refine_state(KrylovState* st, const double* part, int m, int it,
                                                       int every) {
    __shared__ double red[16];
    const double s = block_sum_array(part, m, red);
    if (threadIdx.x == 0) {
        st->conv = 0;
        st->update = 0;
        st->rr0 = s;
        st->it_refine = it;
        st->refine_every = every;
        __hip_atomic_store(&st->done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
void launch_refine_state(KrylovState* st, const double* part, int m, int it, int every, hipStream_t s) {
    k_refine_state<<<1, 1024, 0, s>>>(st, part, m, it, every);
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
void launch_sqnorm_f32_partials(int n, const float* a, double* part, int grid, hipStream_t s) {
    k_sqnorm_f32<<<grid, 256, 0, s>>>(n, a, part);
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
// over chunks of kBjThreads consecutive rows with one row per thread.  A
// chunk's factor entries are first staged in LDS with coalesced loads (up to
// kCap entries; the rest of an unusually dense chunk is read from memory).
// The block's most recent kRing solution values live in an LDS ring (slot =
// local row mod kRing); a slot of the current chunk holds the sentinel until
// its row is final, so a row waits on a same-chunk dependency by re-reading
// the slot.  Dependencies in earlier chunks are final after the chunk barrier
// and are read from the ring, or from global memory once evicted.  No lane
// ever blocks: every pass lets each row consume its terms, in ascending
// column order, up to the first one that is not ready, so the smallest
// pending row always advances.  The solve runs in the factor type F (FP32
// factors: FP32 arithmetic); vectors have type V.
constexpr int kBjThreads = 512;
constexpr int kRing = 4096;
template <typename F> struct BjCap { static constexpr int value = 8192; };
template <> struct BjCap<float> { static constexpr int value = 12288; };

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

// Value of solution entry j.  `cur` tells whether j lies in the current chunk
// (may be pending); `in_ring` whether an earlier row is still in the ring.
template <typename F, typename G>
__device__ __forceinline__ bool fetch_sol(const typename Sentinel<F>::Bits* ring, const G* g, int j, int lo, bool cur,
                                          bool in_ring, F& out) {
    using Bits = typename Sentinel<F>::Bits;
    if (cur) {
        const Bits raw = __hip_atomic_load(&ring[(j - lo) & (kRing - 1)], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        out = from_bits<F>(raw);
        return raw != Sentinel<F>::bits;
    }
    if (in_ring) {
        out = from_bits<F>(ring[(j - lo) & (kRing - 1)]);
        return true;
    }
    out = (F)g[j];
    return true;
}

template <typename V, typename F, int MODE>
__global__ __launch_bounds__(kBjThreads) void k_bj(BJDev P, PcgVecs Vv, KrylovState* st, int it) {
    using Bits = typename Sentinel<F>::Bits;
    constexpr Bits SENT = Sentinel<F>::bits;
    constexpr int kCap = BjCap<F>::value;
    __shared__ Bits ring[kRing];
    __shared__ int scol[kCap];
    __shared__ F sval[kCap];
    __shared__ double red[16];
    __shared__ int shd;
    const int b = blockIdx.x, t = threadIdx.x;
    const int nb = P.nblocks;
    const int lo = P.bp[b], hi = P.bp[b + 1];
    const int* __restrict__ lrp = P.lrp;
    const int* __restrict__ lci = P.lci;
    const F* __restrict__ lval = (const F*)P.lval;
    const int* __restrict__ urp = P.urp;
    const int* __restrict__ uci = P.uci;
    const F* __restrict__ uval = (const F*)P.uval;
    const F* __restrict__ udiag = (const F*)P.udiag;
    V* __restrict__ z = (V*)Vv.z;
    F* __restrict__ y = (F*)Vv.y;
    V* r = (V*)Vv.r;

    if (MODE == 1) {
        if (block_done(st, &shd)) return;
        const double pq = block_sum_array(Vv.part_pq, Vv.npq, red);
        const double rz_old = st->rzs[(it + 1) & 1];
        const double alpha = rz_old / pq;
        if (!(pq > 0.0) || !isfinite(alpha)) {
            if (b == 0 && t == 0) {
                st->breakdown = 1;
                st->iters = it;
                set_done(st);
            }
            return;
        }
        const V a = (V)alpha;
        V* x = (V*)Vv.x;
        const V* p = (const V*)Vv.p;
        const V* q = (const V*)Vv.q;
        double rr = 0.0;
        for (int i = lo + t; i < hi; i += kBjThreads) {
            x[i] = x[i] + a * p[i];
            const V ri = r[i] - a * q[i];
            r[i] = ri;
            rr += (double)ri * (double)ri;
        }
        rr = block_sum(rr, red);
        if (t == 0) Vv.part_rr[b] = rr;
    }
    const V* rin = r;
    int spin_fail = 0;

    // forward substitution: y_i = r_i - sum_{j<i} l_ij y_j.  A chunk is the
    // longest run of at most kBjThreads rows whose entries fit the LDS stage
    // (a single row that does not fit is a chunk of its own and reads its
    // entries from memory; all its dependencies are in earlier chunks).
    // Per row: entries older than the ring (final, in global y) first, then
    // the pass loop, which touches LDS only.  Ascending column order.
    for (int c0 = lo; c0 < hi;) {
        const int ebase = lrp[c0];
        const bool fits = (c0 + t < hi) && (lrp[c0 + t + 1] - ebase <= kCap);
        int nrows = __syncthreads_count(fits);
        const bool big = nrows == 0;
        if (big) nrows = 1;
        const int c1 = c0 + nrows;
        const int nst = big ? 0 : lrp[c1] - ebase;
        for (int e = t; e < nst; e += kBjThreads) {
            scol[e] = lci[ebase + e];
            sval[e] = lval[ebase + e];
        }
        const int i = c0 + t;
        if (i < c1) ring[(i - lo) & (kRing - 1)] = SENT;
        __syncthreads();
        bool fin = i >= c1;
        int pos = fin ? 0 : lrp[i] - ebase;
        const int pend = fin ? 0 : lrp[i + 1] - ebase;
        F acc = fin ? F(0) : (F)rin[i];
        const int ring_lo = c1 - kRing;
        if (!fin && big) {
            // oversized row: every dependency lies in an earlier chunk
            for (; pos < pend; ++pos) {
                const int j = lci[ebase + pos];
                const F yj = (j >= ring_lo) ? from_bits<F>(ring[(j - lo) & (kRing - 1)]) : y[j];
                acc = acc - lval[ebase + pos] * yj;
            }
        }
        if (!fin && ring_lo > lo) {
            // dependencies evicted from the ring: final, read from memory
            while (pos < pend) {
                const int j = scol[pos];
                if (j >= ring_lo) break;
                acc = acc - sval[pos] * y[j];
                ++pos;
            }
        }
        if (!fin) {
            // dependencies in earlier chunks: final, in the ring
            while (pos < pend) {
                const int j = scol[pos];
                if (j >= c0) break;
                acc = acc - sval[pos] * from_bits<F>(ring[(j - lo) & (kRing - 1)]);
                ++pos;
            }
        }
        int spins = 0;
        while (true) {
            if (!fin) {
                // same-chunk dependencies: consume in order up to the first
                // one whose slot still holds the sentinel
                bool blocked = false;
                while (pos < pend && !blocked) {
                    int jj[4];
                    F ww[4];
                    Bits raw[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = min(pos + u, pend - 1);
                        jj[u] = scol[e];
                        ww[u] = sval[e];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        raw[u] = __hip_atomic_load(&ring[(jj[u] - lo) & (kRing - 1)], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool take = !blocked && (pos < pend) && (raw[u] != SENT);
                        const F yv = from_bits<F>(raw[u]);
                        acc = take ? acc - ww[u] * yv : acc;
                        blocked = blocked || !take;
                        pos += take ? 1 : 0;
                    }
                }
                if (pos == pend) {
                    __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<F>(acc), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    fin = true;
                }
            }
            if (__all(fin)) break;
            if (++spins > kSpinLimitIter && !fin) {
                spin_fail = 1;
                __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<F>(acc), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                fin = true;
            }
        }
        __syncthreads();
        if (i < c1) y[i] = from_bits<F>(ring[(i - lo) & (kRing - 1)]);
        __syncthreads();
        c0 = c1;
    }
    // backward substitution: z_i = (y_i - sum_{j>i} u_ij z_j) / u_ii over
    // chunks from the bottom of the block up.  Per row: the pass loop (LDS
    // only) for dependencies still in the ring, then the evicted ones.
    for (int c_hi = hi; c_hi > lo;) {
        const int ebase_hi = urp[c_hi];
        const int rowt = c_hi - 1 - t;
        const bool fits = (t < kBjThreads) && (rowt >= lo) && (ebase_hi - urp[rowt] <= kCap);
        int nrows = __syncthreads_count(fits);
        const bool big = nrows == 0;
        if (big) nrows = 1;
        const int c_lo = c_hi - nrows;
        const int ebase = urp[c_lo];
        const int nst = big ? 0 : ebase_hi - ebase;
        for (int e = t; e < nst; e += kBjThreads) {
            scol[e] = uci[ebase + e];
            sval[e] = uval[ebase + e];
        }
        const int i = c_hi - 1 - t;
        if (i >= c_lo) ring[(i - lo) & (kRing - 1)] = SENT;
        __syncthreads();
        bool fin = i < c_lo;
        int pos = fin ? 0 : urp[i] - ebase;
        const int pend = fin ? 0 : urp[i + 1] - ebase;
        const F dgv = fin ? F(1) : udiag[i];
        F acc = fin ? F(0) : y[i];
        const int ring_hi = c_lo + kRing;
        // same-chunk dependencies (j < c_hi) come first in the row; `lim`
        // marks where the final ones (earlier chunks) start
        int lim = pos;
        if (!fin && !big)
            while (lim < pend && scol[lim] < c_hi) ++lim;
        if (!fin && big) {
            // oversized row: every dependency lies in an earlier chunk
            for (; pos < pend; ++pos) {
                const int j = uci[ebase + pos];
                const F zj = (j < ring_hi) ? from_bits<F>(ring[(j - lo) & (kRing - 1)]) : (F)z[j];
                acc = acc - uval[ebase + pos] * zj;
            }
            lim = pend;
        }
        int spins = 0;
        while (true) {
            if (!fin) {
                bool blocked = false;
                while (pos < lim && !blocked) {
                    int jj[4];
                    F ww[4];
                    Bits raw[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = min(pos + u, lim - 1);
                        jj[u] = scol[e];
                        ww[u] = sval[e];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        raw[u] = __hip_atomic_load(&ring[(jj[u] - lo) & (kRing - 1)], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool take = !blocked && (pos < lim) && (raw[u] != SENT);
                        const F zv = from_bits<F>(raw[u]);
                        acc = take ? acc - ww[u] * zv : acc;
                        blocked = blocked || !take;
                        pos += take ? 1 : 0;
                    }
                }
                if (pos == lim) {
                    // final dependencies of earlier chunks, ascending: in the
                    // ring, then (beyond it) in memory
                    for (; pos < pend; ++pos) {
                        const int j = scol[pos];
                        const F zj = (j < ring_hi) ? from_bits<F>(ring[(j - lo) & (kRing - 1)]) : (F)z[j];
                        acc = acc - sval[pos] * zj;
                    }
                    const F zi = acc / dgv;
                    __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<F>(zi), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    fin = true;
                }
            }
            if (__all(fin)) break;
            if (++spins > kSpinLimitIter && !fin) {
                spin_fail = 1;
                __hip_atomic_store(&ring[(i - lo) & (kRing - 1)], to_bits<F>(acc), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                fin = true;
            }
        }
        __syncthreads();
        if (i >= c_lo) z[i] = (V)from_bits<F>(ring[(i - lo) & (kRing - 1)]);
        __syncthreads();
        c_hi = c_lo;
    }
    if (spin_fail && st) atomicExch(&st->spin_err, 1);
    if (MODE != 0) {
        double rz = 0.0;
        for (int i = lo + t; i < hi; i += kBjThreads) rz += (double)rin[i] * (double)z[i];
        rz = block_sum(rz, red);
        if (t == 0) Vv.part_rz[(it & 1) * nb + b] = rz;
    }
}

template <typename V, typename F>
void launch_bj(int mode, const BJDev& P, const PcgVecs& v, KrylovState* st, int it, hipStream_t s) {
    if (P.nblocks <= 0) return;
    if (mode == 0) k_bj<V, F, 0><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it);
    else if (mode == 1) k_bj<V, F, 1><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it);
    else k_bj<V, F, 2><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it);
}
template void launch_bj<double, double>(int, const BJDev&, const PcgVecs&, KrylovState*, int, hipStream_t);
template void launch_bj<double, float>(int, const BJDev&, const PcgVecs&, KrylovState*, int, hipStream_t);
template void launch_bj<float, float>(int, const BJDev&, const PcgVecs&, KrylovState*, int, hipStream_t);

// ------------------------------------------------------------------ PCG p update
// STEP: convergence test on sum(part_rr) against tol^2 ||b||^2 and the
// refinement trigger (||r||^2 < delta^2 ||r_last||^2), then
// beta = (r,z)_new / (r,z)_old and p = z + beta p.  START: p = z.  REAPPLY:
// the step after a refinement point (no tests).  With a border the
// preconditioned residual is z' = z - W s, s = Kinv (U^T z), and
// (r, z') = (r, z) - t.s, which holds because the block factors of a
// symmetric matrix give a symmetric P.  (r, z') is published in rzs[it & 1].
template <typename T, bool BORDER>
__global__ __launch_bounds__(256) void k_pcg_pupdate(int n, T* __restrict__ p, const T* __restrict__ z,
                                                     const double* __restrict__ part_rz,
                                                     const double* __restrict__ part_rr, int nb, BorderDev bd,
                                                     KrylovState* st, int it, int mode) {
    __shared__ double red[8];
    __shared__ double ts[64];
    __shared__ double ss[64];
    __shared__ int shd;
    if (mode == PUPD_STEP) {
        if (block_done(st, &shd)) return;
        const double rr = block_sum_array(part_rr, nb, red);
        const bool conv = rr <= st->tol2 * st->bb;
        const bool upd = rr < st->delta2 * st->rr0 ||
                         (st->refine_every > 0 && it + 1 - st->it_refine >= st->refine_every);
        if (conv || upd) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->conv = conv ? 1 : 0;
                st->update = upd ? 1 : 0;
                st->iters = it + 1;
                set_done(st);
            }
            return;
        }
    }
    double rz = block_sum_array(part_rz + (it & 1) * nb, nb, red);
    if (BORDER) {
        const int k = bd.k;
        for (int j = threadIdx.x; j < k; j += blockDim.x) {
            double s = 0.0;
            for (int q = 0; q < bd.slices; ++q) s += bd.part[j * bd.slices + q];
            ts[j] = s;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < k; j += blockDim.x) {
            double s = 0.0;
            for (int i = 0; i < k; ++i) s = fma(bd.Kinv[j * k + i], ts[i], s);
            ss[j] = s;
        }
        __syncthreads();
        double ts_dot = 0.0;
        for (int j = 0; j < k; ++j) ts_dot = fma(ts[j], ss[j], ts_dot);
        rz -= ts_dot;
    }
    double beta = 0.0;
    if (mode != PUPD_START) beta = rz / st->rzs[(it + 1) & 1];
    if (!isfinite(beta) || !isfinite(rz)) {
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
    const double* W = bd.W;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        T zi = z[i];
        if (BORDER) {
            double c = 0.0;
            for (int j = 0; j < bd.k; ++j) c = fma(W[(size_t)j * n + i], ss[j], c);
            zi = (T)((double)zi - c);
        }
        p[i] = (mode == PUPD_START) ? zi : zi + bt * p[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rzs[it & 1] = rz;
}

template <typename T>
void launch_pcg_pupdate(int n, const PcgVecs& v, int nblocks, const BorderDev& bd, KrylovState* st, int it,
                        int mode, hipStream_t s) {
    int g = (n + 1023) / 1024;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    if (bd.k > 0)
        k_pcg_pupdate<T, true><<<g, 256, 0, s>>>(n, (T*)v.p, (const T*)v.z, v.part_rz, v.part_rr, nblocks, bd, st,
                                                 it, mode);
    else
        k_pcg_pupdate<T, false><<<g, 256, 0, s>>>(n, (T*)v.p, (const T*)v.z, v.part_rz, v.part_rr, nblocks, bd, st,
                                                  it, mode);
}
template void launch_pcg_pupdate<double>(int, const PcgVecs&, int, const BorderDev&, KrylovState*, int, int,
                                         hipStream_t);
template void launch_pcg_pupdate<float>(int, const PcgVecs&, int, const BorderDev&, KrylovState*, int, int,
                                        hipStream_t);

// z <- z - W s, s = Kinv (sum of the U^T z partials): the border correction
// on its own (the solve loop fuses it into the direction update)
template <typename T>
__global__ __launch_bounds__(256) void k_border_fix(int n, T* __restrict__ z, BorderDev bd) {
    __shared__ double ts[64];
    __shared__ double ss[64];
    const int k = bd.k;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < bd.slices; ++q) s += bd.part[j * bd.slices + q];
        ts[j] = s;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s = fma(bd.Kinv[j * k + i], ts[i], s);
        ss[j] = s;
    }
    __syncthreads();
    const double* W = bd.W;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double c = 0.0;
        for (int j = 0; j < k; ++j) c = fma(W[(size_t)j * n + i], ss[j], c);
        z[i] = (T)((double)z[i] - c);
    }
}
template <typename T>
void launch_border_fix(int n, T* z, const BorderDev& bd, hipStream_t s) {
    if (bd.k <= 0) return;
    const int g = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
    k_border_fix<T><<<g > 0 ? g : 1, 256, 0, s>>>(n, z, bd);
}
template void launch_border_fix<double>(int, double*, const BorderDev&, hipStream_t);
template void launch_border_fix<float>(int, float*, const BorderDev&, hipStream_t);

// ------------------------------------------------------------------ border setup
__global__ void k_scatter_column(int n, const int* __restrict__ ucp, const int* __restrict__ uri,
                                 const double* __restrict__ ucv, int j, double* __restrict__ e) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) e[i] = 0.0;
}
__global__ void k_scatter_column2(const int* __restrict__ ucp, const int* __restrict__ uri,
                                  const double* __restrict__ ucv, int j, double* __restrict__ e) {
    for (int p = ucp[j] + blockIdx.x * blockDim.x + threadIdx.x; p < ucp[j + 1]; p += gridDim.x * blockDim.x)
        e[uri[p]] = ucv[p];
}
void launch_scatter_column(int n, const int* ucp, const int* uri, const double* ucv, int j, double* e,
                           hipStream_t s) {
    const int g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    k_scatter_column<<<g > 0 ? g : 1, 256, 0, s>>>(n, ucp, uri, ucv, j, e);
    k_scatter_column2<<<256, 256, 0, s>>>(ucp, uri, ucv, j, e);
}

// K[a][b] = (a == b ? 1 / c_a : 0) + sum_{i in col a} U_ia W_ib, one workgroup per entry
__global__ __launch_bounds__(256) void k_border_k(int n, int k, const int* __restrict__ ucp,
                                                  const int* __restrict__ uri, const double* __restrict__ ucv,
                                                  const double* __restrict__ c, const double* __restrict__ W,
                                                  double* __restrict__ K) {
    __shared__ double red[8];
    const int a = blockIdx.x / k, b = blockIdx.x % k;
    double s = 0.0;
    for (int p = ucp[a] + threadIdx.x; p < ucp[a + 1]; p += blockDim.x) s = fma(ucv[p], W[(size_t)b * n + uri[p]], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) K[a * k + b] = s + (a == b ? 1.0 / c[a] : 0.0);
}
void launch_border_k(int n, int k, const int* ucp, const int* uri, const double* ucv, const double* c,
                     const double* W, double* K, hipStream_t s) {
    k_border_k<<<k * k, 256, 0, s>>>(n, k, ucp, uri, ucv, c, W, K);
}

// Kinv = K^{-1} for k <= 64 by Gauss-Jordan elimination with partial
// pivoting in LDS (one workgroup).  status = 1 on a zero pivot.
__global__ __launch_bounds__(64) void k_small_inverse(int k, const double* __restrict__ K, double* __restrict__ Kinv,
                                                      int* status) {
    __shared__ double A[64][129];
    __shared__ int piv;
    const int t = threadIdx.x;
    for (int i = 0; i < k; ++i) {
        if (t < k) {
            A[i][t] = K[i * k + t];
            A[i][k + t] = (i == t) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    int bad = 0;
    for (int col = 0; col < k; ++col) {
        if (t == 0) {
            int pr = col;
            double best = fabs(A[col][col]);
            for (int i = col + 1; i < k; ++i)
                if (fabs(A[i][col]) > best) { best = fabs(A[i][col]); pr = i; }
            piv = pr;
        }
        __syncthreads();
        const int pr = piv;
        if (pr != col)
            for (int j = t; j < 2 * k; j += 64) { const double tmp = A[col][j]; A[col][j] = A[pr][j]; A[pr][j] = tmp; }
        __syncthreads();
        const double d = A[col][col];
        if (d == 0.0) { bad = 1; break; }
        for (int j = t; j < 2 * k; j += 64) A[col][j] = A[col][j] / d;
        __syncthreads();
        for (int i = 0; i < k; ++i) {
            if (i == col) continue;
            const double f = A[i][col];
            __syncthreads();
            for (int j = t; j < 2 * k; j += 64) A[i][j] = fma(-f, A[col][j], A[i][j]);
            __syncthreads();
        }
    }
    if (t == 0) *status = bad;
    if (!bad)
        for (int i = 0; i < k; ++i)
            if (t < k) Kinv[i * k + t] = A[i][k + t];
}
void launch_small_inverse(int k, const double* K, double* Kinv, int* status, hipStream_t s) {
    k_small_inverse<<<1, 64, 0, s>>>(k, K, Kinv, status);
}

}  // namespace sdsl
