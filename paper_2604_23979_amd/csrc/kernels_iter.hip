// Per-iteration kernels on gfx950: CSR SpMV with fused dot, compensated FP64
// residual, the block-Jacobi apply (forward + backward substitution of every
// block in one launch, fused with the PCG vector updates) and the PCG
// direction update.
#include "common.hpp"

namespace sdsl {


// ------------------------------------------------------------------ helpers
// Reads typed by address space.  A value that comes from LDS on one path and
// from global memory on another is otherwise read by one merged flat load,
// and waiting for a flat load waits for every load in flight (those issued
// ahead on purpose); loads of different address spaces are never merged.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ T lload(const T* p) {
    return *(const __attribute__((address_space(3))) T*)p;
}

__device__ __forceinline__ bool krylov_done(const KrylovState* st) {
    return __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// TwoSum (Knuth): s = fl(a + b) and e = (a + b) - s exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

// Workgroup sum of (s, e) pairs in which every addition is a TwoSum whose
// error joins e, so that s + e keeps the rounding of each step; the result
// is in thread 0.  `scratch` holds >= 2 * blockDim.x / 64 doubles.  Must be
// reached by all threads.
__device__ __forceinline__ void block_sum2(double& s, double& e, double* scratch) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double so = __shfl_xor(s, o, kWave), eo = __shfl_xor(e, o, kWave);
        double t, te;
        two_sum(s, so, t, te);
        s = t;
        e = e + eo + te;
    }
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (l == 0) {
        scratch[w] = s;
        scratch[nw + w] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = scratch[0], e0 = scratch[nw];
        for (int q = 1; q < nw; ++q) {
            double t, te;
            two_sum(t0, scratch[q], t, te);
            t0 = t;
            e0 = e0 + scratch[nw + q] + te;
        }
        s = t0;
        e = e0;
    }
    __syncthreads();
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
    // about kSpmvRows rows per workgroup, but no more than two workgroups per
    // CU (512) while a workgroup stays within kSpmvMaxRows rows, so that a
    // large SpMV runs as one wave of resident workgroups; a multiple of 8 so
    // that the XCD swizzle is a permutation (the extra workgroups have no
    // rows)
    int g = (n + kSpmvRows - 1) / kSpmvRows;
    g = std::min(g, std::max(512, (n + kSpmvMaxRows - 1) / kSpmvMaxRows));
    g = (g + 7) / 8 * 8;
    return g < 8 ? 8 : g;
}

// rows per SpMV workgroup for a grid: a multiple of 16 (one share per wave)
int spmv_rows(int n, int grid) {
    int r = (n + grid - 1) / grid;
    r = (r + 15) / 16 * 16;
    return r < 16 ? 16 : r;
}

// lanes per row of the SpMV (4 loads per lane per round): the smallest
// power of two from 4 to 64 whose round covers the mean row
int spmv_lanes(double mean_row) {
    int g = 4;
    while (g < 64 && 4 * g < mean_row) g *= 2;
    return g;
}

// ------------------------------------------------------------------ low rank
// part[j * slices + s] = sum over slice s of column j of U^T x (FP64).  With
// COMP the slice sums are compensated and their error terms go to
// part[k * slices + j * slices + s].  With FOLD = LR_SCALED the last
// workgroup to finish sums the slices of every column in slice order and
// writes c_j (U^T x)_j into lr.fold, so that the SpMV reads k values instead
// of k * slices; with LR_BORDER the consumers fold the partials themselves
// (LrFold).
template <typename T, bool COMP, int FOLD>
__global__ __launch_bounds__(256) void k_lowrank_tdot(LowRankDev lr, const T* __restrict__ x,
                                                      const KrylovState* st) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const int k = lr.k, slices = lr.slices;
    const int* __restrict__ uri = lr.uri;
    const double* __restrict__ ucv = (const double*)lr.ucv;
    double* part = lr.part;
    const int j = blockIdx.x / slices, s = blockIdx.x % slices;
    const int a = lr.ucp[j], e = lr.ucp[j + 1];
    const int len = e - a;
    const int lo = a + (int)((int64_t)len * s / slices), hi = a + (int)((int64_t)len * (s + 1) / slices);
    double sum = 0.0, err = 0.0;
    // four strides of loads in flight per thread; each thread still adds its
    // entries in ascending order
    for (int p0 = lo + (int)threadIdx.x; p0 < hi; p0 += 4 * (int)blockDim.x) {
        int id[4];
        double uv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = p0 + u * (int)blockDim.x;
            id[u] = p < hi ? uri[p] : 0;
            uv[u] = p < hi ? ucv[p] : 0.0;
        }
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = (p0 + u * (int)blockDim.x < hi) ? (double)x[id[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (p0 + u * (int)blockDim.x >= hi) break;
            const double pr = uv[u] * xv[u];
            if (COMP) {
                const double pe = fma(uv[u], xv[u], -pr);
                const double t = sum + pr;
                const double z = t - sum;
                err += (sum - (t - z)) + (pr - z) + pe;
                sum = t;
            } else {
                sum += pr;
            }
        }
    }
    if (COMP) {
        // the thread pairs combine with TwoSum as well: under the cancellation
        // of a converged residual, a plain sum of the thread sums would lose
        // more than the residual itself once c_j is large
        block_sum2(sum, err, red);
        if (threadIdx.x == 0) {
            part[j * slices + s] = sum;
            part[k * slices + j * slices + s] = err;
        }
    } else {
        const double tot = block_sum(sum, red);
        if (threadIdx.x == 0) part[j * slices + s] = tot;
    }
    if (FOLD == LR_SCALED) {
        __shared__ double sp[kMaxRank * kMaxRank];
        __shared__ int last;
        if (threadIdx.x == 0) {
            __threadfence();  // publish this workgroup's partial
            const unsigned prev = atomicInc(lr.counter, gridDim.x - 1);
            last = prev == gridDim.x - 1;
        }
        __syncthreads();
        if (!last) return;
        __threadfence();  // every partial is visible
        const int m = k * slices;
        for (int q = threadIdx.x; q < m; q += blockDim.x) sp[q] = part[q];
        __syncthreads();
        for (int jj = threadIdx.x; jj < k; jj += blockDim.x) {
            double t = 0.0;
            for (int q = 0; q < slices; ++q) t += sp[jj * slices + q];
            lr.fold[jj] = ((const double*)lr.c)[jj] * t;
        }
    }
}

template <typename T>
void launch_lowrank_tdot(const LowRankDev& lr, const T* x, const KrylovState* st, int fold, hipStream_t s) {
    if (lr.k <= 0) return;
    const int g = lr.k * lr.slices;
    if (fold == LR_SCALED) k_lowrank_tdot<T, false, LR_SCALED><<<g, 256, 0, s>>>(lr, x, st);
    else if (fold == LR_BORDER) k_lowrank_tdot<T, false, LR_BORDER><<<g, 256, 0, s>>>(lr, x, st);
    else k_lowrank_tdot<T, false, LR_NONE><<<g, 256, 0, s>>>(lr, x, st);
}
template void launch_lowrank_tdot<double>(const LowRankDev&, const double*, const KrylovState*, int, hipStream_t);
template void launch_lowrank_tdot<float>(const LowRankDev&, const float*, const KrylovState*, int, hipStream_t);

// ------------------------------------------------------------------ SpMV
// y = M x (+ U diag(c) U^T x) with G lanes per row.  Values (type F) and
// column indices are streamed with non-temporal loads so that the gathered x
// (type V) stays in L2; the products and their sum are formed in F (FP32
// values give an FP32 product, accumulated in FP32); the low-rank term is
// added in FP64.  With part_dot the workgroup's share of (x, y) is written
// to part_dot[w].
//
// Layout of the launch: a workgroup of kSpmvThreads threads owns `rows`
// consecutive rows (spmv_rows; XCD-swizzled); each of its waves takes
// rows / 16 of them, 64 / G rows per step with G lanes per row and U
// loads per lane per round, and the loads of the next step are issued before
// the current step gathers x.  Row sums use DPP lane exchanges (no LDS).
//
// Near window: with halo > 0 the workgroup first copies x[r0 - halo,
// r1 + halo) (rounded to F) into LDS; entries whose column falls inside are
// gathered from LDS, the others from memory.  Banded-plus-scattered
// patterns keep most gathers off the L2.

// v moved by DPP control CTRL within the enabled rows (others give 0)
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    int lo = (int)(b & 0xffffffff), hi = (int)(b >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWM, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWM, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ float dpp_move(float v) {
    const int b = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWM, 0xF, false);
    return __builtin_bit_cast(float, b);
}
// Sum over aligned groups of G lanes.  The total is valid in every lane of
// the group for G <= 16, in lanes 16..31 of each 32-lane group for G = 32
// and in lanes 48..63 for G = 64 (kSumLane<G> is the first such lane).
template <int G, typename T>
__device__ __forceinline__ T dpp_sum(T s) {
    if (G >= 2) s += dpp_move<0xB1>(s);        // quad_perm [1,0,3,2]
    if (G >= 4) s += dpp_move<0x4E>(s);        // quad_perm [2,3,0,1]
    if (G >= 8) s += dpp_move<0x141>(s);       // row_half_mirror
    if (G >= 16) s += dpp_move<0x140>(s);      // row_mirror
    if (G >= 32) s += dpp_move<0x142, 0xA>(s); // row_bcast:15 into rows 1, 3
    if (G >= 64) s += dpp_move<0x143, 0xC>(s); // row_bcast:31 into rows 2, 3
    return s;
}
template <int G> struct SumLane { static constexpr int value = G <= 16 ? 0 : (G == 32 ? 16 : 48); };

template <typename V, typename F, int G, int U, bool LR>
__device__ __forceinline__ void spmv_body(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                          const F* __restrict__ v, const V* __restrict__ x, V* __restrict__ y,
                                          double* __restrict__ part_dot, const KrylovState* st, LowRankDev lr,
                                          int halo, int rows, int bid, int gdim) {
    extern __shared__ double xwin_lds[];
    __shared__ double red[16];
    __shared__ double tk[kMaxRank];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    if (LR) {
        for (int j = threadIdx.x; j < lr.k; j += blockDim.x) tk[j] = lr.fold[j];
    }
    const int g = gdim;
    const int lw = xcd_swizzle(bid, g);
    const int r0 = min(n, lw * rows), r1 = min(n, r0 + rows);
    F* xs = reinterpret_cast<F*>(xwin_lds);
    const int wlo = halo > 0 ? max(0, r0 - halo) : 0;
    const int whi = halo > 0 ? min(n, r1 + halo) - 1 : -1;  // empty window without halo
    for (int c0 = wlo + (int)threadIdx.x; c0 <= whi; c0 += 4 * kSpmvThreads) {
        V t4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * kSpmvThreads;
            t4[u] = c <= whi ? x[c] : V(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * kSpmvThreads;
            if (c <= whi) xs[c - wlo] = (F)t4[u];
        }
    }
    __syncthreads();
    // x_c comes from the window (LDS) or from memory, each read in its own
    // address space (one merged flat read would wait for every load in
    // flight); a round's terms are added window terms first, then memory
    // terms, each in slot order
    auto in_win = [&](int c) { return c >= wlo && c <= whi; };

    constexpr int RPS = kWave / G;
    const int RW = rows / (kSpmvThreads / kWave);  // rows per wave (at most 64)
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int grp = lane / G, gl = lane % G;
    const int base = r0 + wave * RW;
    const int nrow = max(0, min(RW, r1 - base));
    double dacc = 0.0;
    if (nrow > 0) {
        const int my_a = lane < nrow ? rp[base + lane] : 0;
        const int my_e = lane < nrow ? rp[base + lane + 1] : 0;
        int my_u0 = 0, my_u1 = 0;
        if (LR) {
            my_u0 = lane < nrow ? lr.urp[base + lane] : 0;
            my_u1 = lane < nrow ? lr.urp[base + lane + 1] : 0;
        }
        F vv[U], nv[U];
        int cc[U], nc[U];
        int a = __shfl(my_a, grp, kWave), e = __shfl(my_e, grp, kWave);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = a + gl + u * G;
            vv[u] = p < e ? __builtin_nontemporal_load(&v[p]) : F(0);
            cc[u] = p < e ? __builtin_nontemporal_load(&ci[p]) : r0;
        }
        // low-rank entries of a step's rows (first G of each row), loaded one
        // step ahead like the operator's entries
        auto lr_load = [&](int j, double& w, int& c) {
            w = 0.0;
            c = 0;
            if (LR && j < nrow) {
                const int row_j = min(j + grp, nrow - 1);
                const int ua = __shfl(my_u0, row_j, kWave), ue = __shfl(my_u1, row_j, kWave);
                if (j + grp < nrow && ua + gl < ue) {
                    w = ((const double*)lr.uv)[ua + gl];
                    c = lr.uci[ua + gl];
                }
            }
        };
        double lw = 0.0, nlw = 0.0;
        int lc = 0, nlc = 0;
        lr_load(0, lw, lc);
        for (int j = 0; j < nrow; j += RPS) {
            // next step's entries in flight while this one gathers
            const int jn = j + RPS;
            const int an = __shfl(my_a, min(jn + grp, kWave - 1), kWave);
            const int en = __shfl(my_e, min(jn + grp, kWave - 1), kWave);
            const bool more = jn < nrow;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = an + gl + u * G;
                const bool ok = more && p < en;
                nv[u] = ok ? __builtin_nontemporal_load(&v[p]) : F(0);
                nc[u] = ok ? __builtin_nontemporal_load(&ci[p]) : r0;
            }
            lr_load(jn, nlw, nlc);
            F s = F(0);
            {
                V m[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    m[u] = V(0);
                    if (!in_win(cc[u])) m[u] = gload(x + cc[u]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (in_win(cc[u])) s = fma(vv[u], lload(xs + (cc[u] - wlo)), s);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (!in_win(cc[u])) s = fma(vv[u], (F)m[u], s);
            }
            // rows longer than one round, entry by entry
            for (int p0 = a + gl + U * G; p0 < e; p0 += U * G) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int p = p0 + u * G;
                    if (p < e) {
                        const int c = ci[p];
                        const F w = in_win(c) ? lload(xs + (c - wlo)) : F(0);
                        const V m = in_win(c) ? V(0) : gload(x + c);
                        s = fma(v[p], in_win(c) ? w : (F)m, s);
                    }
                }
            }
            // low-rank term of the step's rows, FP64, one entry per lane
            double t = 0.0;
            if (LR) {
                t = lw * tk[lc];
                const int row_j = min(j + grp, nrow - 1);
                const int ua = __shfl(my_u0, row_j, kWave), ue = __shfl(my_u1, row_j, kWave);
                for (int q = ua + gl + G; q < ue; q += G)
                    t = fma(((const double*)lr.uv)[q], tk[lr.uci[q]], t);
            }
            s = dpp_sum<G>(s);
            if (LR) t = dpp_sum<G>(t);
            const int row = j + grp;
            if (gl == SumLane<G>::value && row < nrow) {
                const V out = LR ? (V)((double)s + t) : (V)s;
                y[base + row] = out;
                if (part_dot) dacc += (double)gload(x + base + row) * (double)out;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                vv[u] = nv[u];
                cc[u] = nc[u];
            }
            lw = nlw;
            lc = nlc;
            a = an;
            e = en;
        }
    }
    if (part_dot) {
        const double tot = block_sum(dacc, red);
        if (threadIdx.x == 0) part_dot[bid] = tot;
    }
}
template <typename V, typename F, int G, int U, bool LR>
__global__ __launch_bounds__(kSpmvThreads, 8) void k_spmv(int n, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const F* __restrict__ v,
                                                       const V* __restrict__ x, V* __restrict__ y,
                                                       double* __restrict__ part_dot, const KrylovState* st,
                                                       LowRankDev lr, int halo, int rows) {
    spmv_body<V, F, G, U, LR>(n, rp, ci, v, x, y, part_dot, st, lr, halo, rows, blockIdx.x, gridDim.x);
}


// Entries of the SpMV workgroups' rows whose column lies in the near window
// [r0 - halo, r1 + halo): count[0] += their number.
__global__ __launch_bounds__(256) void k_spmv_near(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   int halo, int rows, unsigned long long* count) {
    const int w = blockIdx.x;
    const int r0 = min(n, w * rows), r1 = min(n, r0 + rows);
    const int lo = max(0, r0 - halo), hi = min(n, r1 + halo);
    unsigned long long c = 0;
    for (int p = rp[r0] + (int)threadIdx.x; p < rp[r1]; p += blockDim.x) c += (ci[p] >= lo && ci[p] < hi);
    atomicAdd(count, c);
}
void launch_spmv_near(int n, int grid, const int* rp, const int* ci, int halo, unsigned long long* count,
                      hipStream_t s) {
    k_spmv_near<<<grid, 256, 0, s>>>(n, rp, ci, halo, spmv_rows(n, grid), count);
}

template <typename V, typename F, bool LR>
static void spmv_dispatch(const CsrView& A, const F* v, const LowRankDev& lr, const V* x, V* y, double* pd,
                          const KrylovState* st, int lanes, int grid, hipStream_t s) {
    const int rows = spmv_rows(A.n, grid);
    const size_t shm = A.halo > 0 ? (size_t)(rows + 2 * A.halo) * sizeof(F) : 0;
    constexpr int T = kSpmvThreads;
    switch (lanes) {
        case 64: k_spmv<V, F, 64, 4, LR><<<grid, T, shm, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr, A.halo, rows); break;
        case 32: k_spmv<V, F, 32, 4, LR><<<grid, T, shm, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr, A.halo, rows); break;
        case 16: k_spmv<V, F, 16, 4, LR><<<grid, T, shm, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr, A.halo, rows); break;
        case 8: k_spmv<V, F, 8, 4, LR><<<grid, T, shm, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr, A.halo, rows); break;
        default: k_spmv<V, F, 4, 4, LR><<<grid, T, shm, s>>>(A.n, A.rp, A.ci, v, x, y, pd, st, lr, A.halo, rows); break;
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
        k_lowrank_tdot<double, true, LR_NONE><<<lr.k * lr.slices, 256, 0, s>>>(lr, x, nullptr);
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

// ------------------------------------------------------------------ MC64 transform
// Alg. 3 (Sec. 3.3) on the device, with the matching and scalings found at
// setup: values of A' = Q Dr A Dc from new values of A (entry p of A goes to
// position emap[p] of A', times escale[p] = dr_row * dc_col), the
// right-hand side b' = Q Dr b (b'_k = rs_k b_{rowof_k}) and the solution
// x = Dc y.
__global__ void k_mc64_values(int64_t nnz, const int* __restrict__ emap, const double* __restrict__ escale,
                              const double* __restrict__ a, double* __restrict__ out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        out[emap[p]] = escale[p] * a[p];
}
void launch_mc64_values(int64_t nnz, const int* emap, const double* escale, const double* a, double* out,
                        hipStream_t s) {
    const int64_t g = (nnz + 255) / 256;
    if (nnz > 0) k_mc64_values<<<(int)(g < 4096 ? g : 4096), 256, 0, s>>>(nnz, emap, escale, a, out);
}
__global__ void k_mc64_rhs(int n, const int* __restrict__ rowof, const double* __restrict__ rs,
                           const double* __restrict__ b, double* __restrict__ out) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) out[k] = rs[k] * b[rowof[k]];
}
void launch_mc64_rhs(int n, const int* rowof, const double* rs, const double* b, double* out, hipStream_t s) {
    const int g = std::min(4096, (n + 255) / 256);
    if (n > 0) k_mc64_rhs<<<g, 256, 0, s>>>(n, rowof, rs, b, out);
}
__global__ void k_mc64_sol(int n, const double* __restrict__ cs, const double* __restrict__ y,
                           double* __restrict__ x) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) x[j] = cs[j] * y[j];
}
void launch_mc64_sol(int n, const double* cs, const double* y, double* x, hipStream_t s) {
    const int g = std::min(4096, (n + 255) / 256);
    if (n > 0) k_mc64_sol<<<g, 256, 0, s>>>(n, cs, y, x);
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

// ------------------------------------------------------------------ GMRES
// Arnoldi building blocks (Sec. 2.2, GMRES with right preconditioning).
// Basis vectors are columns of V (n x k, column c at V + c * ldv).
constexpr int kMaxBasis = 64;       // k <= kMaxBasis columns per call
constexpr int kDotGrid = 512;       // workgroups of the multi-dot pass

// part[w * kMaxBasis + c] = workgroup w's share of (V_c, w), c < k
__global__ __launch_bounds__(256) void k_multidot(int n, int k, const double* __restrict__ V, int64_t ldv,
                                                  const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double red[kMaxBasis][4];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int c0 = 0; c0 < k; c0 += 16) {
        double acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const double wi = w[i];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (c0 + u < k) acc[u] = fma(V[(int64_t)(c0 + u) * ldv + i], wi, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const double s = wave_sum(acc[u]);
            if (lane == 0 && c0 + u < k) red[c0 + u][wave] = s;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x)
        part[(int64_t)blockIdx.x * kMaxBasis + c] = ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3];
}
// out[c] = sum over the grid of part[. * kMaxBasis + c] (fixed order); with
// acc, acc[c] += out[c] as well
__global__ __launch_bounds__(kMaxBasis) void k_multidot_reduce(int k, int grid, const double* __restrict__ part,
                                                               double* __restrict__ out, double* acc) {
    const int c = threadIdx.x;
    if (c >= k) return;
    double s = 0.0;
    for (int w0 = 0; w0 < grid; w0 += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = w0 + u < grid ? part[(int64_t)(w0 + u) * kMaxBasis + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    out[c] = s;
    if (acc) acc[c] += s;
}
void launch_multidot(int n, int k, const double* V, int64_t ldv, const double* w, double* part, double* out,
                     double* acc, hipStream_t s) {
    k_multidot<<<kDotGrid, 256, 0, s>>>(n, k, V, ldv, w, part);
    k_multidot_reduce<<<1, kMaxBasis, 0, s>>>(k, kDotGrid, part, out, acc);
}

// w += alpha * sum_c V_c coef[c] (coef on the device); with nrm_part the
// workgroup's share of ||w||^2 after the update goes to nrm_part[w]
__global__ __launch_bounds__(256) void k_multiaxpy(int n, int k, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ coef, double alpha,
                                                   double* __restrict__ w, double* __restrict__ nrm_part) {
    __shared__ double cf[kMaxBasis];
    __shared__ double red[8];
    for (int c = threadIdx.x; c < k; c += blockDim.x) cf[c] = alpha * coef[c];
    __syncthreads();
    double sq = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int c = 0; c < k; ++c) t = fma(V[(int64_t)c * ldv + i], cf[c], t);
        const double wi = w[i] + t;
        w[i] = wi;
        sq = fma(wi, wi, sq);
    }
    if (nrm_part) {
        const double tot = block_sum(sq, red);
        if (threadIdx.x == 0) nrm_part[blockIdx.x] = tot;
    }
}
void launch_multiaxpy(int n, int k, const double* V, int64_t ldv, const double* coef, double alpha, double* w,
                      double* nrm_part, hipStream_t s) {
    k_multiaxpy<<<kDotGrid, 256, 0, s>>>(n, k, V, ldv, coef, alpha, w, nrm_part);
}
// v = w / sqrt(*nrm2)
__global__ void k_scale_inv_norm(int n, const double* __restrict__ nrm2, const double* __restrict__ w,
                                 double* __restrict__ v) {
    const double inv = 1.0 / sqrt(nrm2[0]);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = w[i] * inv;
}
void launch_scale_inv_norm(int n, const double* nrm2, const double* w, double* v, hipStream_t s) {
    const int g = std::min(4096, (n + 255) / 256);
    k_scale_inv_norm<<<std::max(g, 1), 256, 0, s>>>(n, nrm2, w, v);
}

// ------------------------------------------------------------------ BJ apply
// One workgroup per diagonal block (all blocks in one launch).  Forward
// substitution y = L^{-1} r then backward substitution z = U^{-1} y, each
// over chunks of kBjThreads consecutive rows, one row per thread: forward
// chunks are cut from the top of the block, backward chunks from the bottom.
// The level of every row inside its chunk is fixed by the factor's pattern
// and built once per factorisation (k_bj_levels).
// Factor entries: the newest kEll entries of a row (those nearest the
// diagonal) sit in a chunk-interleaved copy (k_bj_ell) that is read with
// coalesced loads straight into registers one chunk ahead; the older
// entries of longer rows sit in a CSR of their own whose range for a whole
// chunk is contiguous, and are staged into LDS with coalesced loads, also
// one chunk ahead.
// The block's most recent solution values live in an LDS ring (slot = local
// row mod ring size); older values are read from memory.  At the start of a
// chunk every row subtracts, in one straight pass, its terms on earlier
// chunks (all final); the same-chunk terms wait for the row's level: levels
// are separated by workgroup barriers, so at its level every term of a row
// is final.  Those terms are prepared at the start of the chunk as (ring
// offset, weight) pairs, so that a level runs without branches; unused
// pairs point at a zero slot with a zero weight, which leaves the sum
// unchanged.  Terms are subtracted in the order of a plain substitution
// (forward: ascending columns, backward: descending), each with a separate
// product and difference.  The solve runs in the factor type F (FP32
// factors: FP32 arithmetic); vectors have type V.
constexpr int kEll = kBjEllWidth;
static_assert(kEll % 4 == 0, "the straight pass reads ELL slots four at a time");
constexpr int kHeld = 8;                   // newest slots kept in registers through the levels
constexpr int kPark = kEll - kHeld;        // the others, parked in LDS
constexpr int kStageOld = 2 * kBjThreads;  // older entries of a chunk staged in LDS
// solution values kept in LDS per block (FP64 solves leave room for the
// parked FP64 weights)
template <typename F>
struct BjRing {
    static constexpr int size = sizeof(F) == 8 ? 4096 : 8192;
};

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

// Rows [ca, cb) of sweep chunk m of the block [lo, hi).
template <bool FWD>
__device__ __forceinline__ void bj_chunk(int lo, int hi, int m, int& ca, int& cb) {
    if (FWD) {
        ca = lo + m * kBjThreads;
        cb = min(hi, ca + kBjThreads);
    } else {
        cb = hi - m * kBjThreads;
        ca = max(lo, cb - kBjThreads);
    }
}

// Chunk tables of block b in the layout k_bj_levels reads, both with room
// for hi - lo + 1 entries at offset lo + b: lch[m] = {first row of forward
// chunk m, lrp[that row]}, lch[nch] = {hi, lrp[hi]}; uch[m] = {end row of
// backward chunk m, urp[that row]} from {hi, urp[hi]} down to {lo, urp[lo]}.
__global__ __launch_bounds__(256) void k_bj_chunks(const int* __restrict__ bp, const int* __restrict__ lrp,
                                                   const int* __restrict__ urp, int2* __restrict__ lch,
                                                   int2* __restrict__ uch) {
    const int b = blockIdx.x;
    const int lo = bp[b], hi = bp[b + 1];
    const int nch = (hi - lo + kBjThreads - 1) / kBjThreads;
    for (int m = threadIdx.x; m <= nch; m += blockDim.x) {
        const int a = min(hi, lo + m * kBjThreads);
        lch[lo + b + m] = make_int2(a, lrp[a]);
        const int e = max(lo, hi - m * kBjThreads);
        uch[lo + b + m] = make_int2(e, urp[e]);
    }
}
void launch_bj_chunks(int nblocks, const int* bp, const int* lrp, const int* urp, int2* lch, int2* uch,
                      hipStream_t s) {
    if (nblocks > 0) k_bj_chunks<<<nblocks, 256, 0, s>>>(bp, lrp, urp, lch, uch);
}

// Local levels of the rows of every chunk: level(i) = 0 if row i has no
// dependency inside its chunk, else 1 + the largest level among them, so a
// chunk is solved level by level with a barrier in between and every term
// a row takes is final.  llev/ulev hold the level per row, lnl/unl the
// number of levels per chunk (same indexing as the chunk tables).  Computed
// in rounds: a row gets its level once all its same-chunk dependencies have
// one; a chain of r rows needs r rounds and at most nrows rounds are run.
// The sweeps give the rows of a chunk to threads grouped by how many ELL
// slots they occupy and in level order inside a group, so that the rows of
// one level share a few wavefronts and the cache lines of a slot mostly
// serve rows that occupy it: lperm/uperm hold, at the chunk's first row + p,
// {the row solved by thread p, its number of entries}, and lpos/upos the
// inverse.
__global__ __launch_bounds__(kBjThreads) void k_bj_levels(const int* __restrict__ bp, const int* __restrict__ lrp,
                                                          const int* __restrict__ lci, const int* __restrict__ urp,
                                                          const int* __restrict__ uci, const int2* __restrict__ lch,
                                                          const int2* __restrict__ uch, int* __restrict__ llev,
                                                          int* __restrict__ ulev, int* __restrict__ lnl,
                                                          int* __restrict__ unl, int2* __restrict__ lperm,
                                                          int2* __restrict__ uperm, int* __restrict__ lpos,
                                                          int* __restrict__ upos) {
    __shared__ int slev[kBjThreads];
    __shared__ int slen[kBjThreads];
    __shared__ int smax;
    const int b = blockIdx.x, t = threadIdx.x;
    const int lo = bp[b], hi = bp[b + 1];
    const int2* L = lch + lo + b;
    const int2* U = uch + lo + b;
    for (int dir = 0; dir < 2; ++dir) {
        const int2* T = dir == 0 ? L : U;
        const int* rp = dir == 0 ? lrp : urp;
        const int* ci = dir == 0 ? lci : uci;
        int* lev = dir == 0 ? llev : ulev;
        int2* perm = dir == 0 ? lperm : uperm;
        int* pos = dir == 0 ? lpos : upos;
        int* nl = (dir == 0 ? lnl : unl) + lo + b;
        const int end = dir == 0 ? hi : lo;
        for (int m = 0; T[m].x != end; ++m) {
            // chunk rows: forward [a, e) with row a + t; backward [e, a) with row a - 1 - t
            const int a = T[m].x, e = T[m + 1].x;
            const int nrows = dir == 0 ? e - a : a - e;
            const int i = dir == 0 ? a + t : a - 1 - t;
            const bool live = t < nrows;
            // same-chunk dependencies: the tail of the row in both directions
            // (forward rows ascend, j >= a; backward rows descend, j < a)
            int q0 = 0, q1 = 0, rlen = 0;
            if (live) {
                q0 = rp[i];
                q1 = rp[i + 1];
                rlen = q1 - q0;
                int f = q1;
                if (dir == 0)
                    while (f > q0 && ci[f - 1] >= a) --f;
                else
                    while (f > q0 && ci[f - 1] < a) --f;
                q0 = f;
            }
            slev[t] = -1;
            if (t == 0) smax = 0;
            __syncthreads();
            int mine = live ? -1 : 0;
            for (int round = 0; round <= nrows; ++round) {
                if (mine < 0) {
                    int mx = -1;
                    bool ok = true;
                    for (int q = q0; q < q1 && ok; ++q) {
                        const int j = ci[q];
                        const int pj = dir == 0 ? j - a : a - 1 - j;
                        const int lj = __hip_atomic_load(&slev[pj], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        ok = lj >= 0;
                        mx = lj > mx ? lj : mx;
                    }
                    if (ok) {
                        mine = mx + 1;
                        __hip_atomic_store(&slev[t], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                if (__syncthreads_count(mine < 0) == 0) break;
            }
            slen[t] = min(rlen, kEll);  // occupied ELL slots
            if (live) {
                lev[i] = mine;
                atomicMax(&smax, mine + 1);
            }
            __syncthreads();
            if (t == 0) nl[m] = smax;
            if (live) {
                // place in the chunk: rows by occupied ELL slots in groups
                // of eight (17-24 first, then 9-16, 1-8, none), each group in
                // level order, then row order (the same in every setup): a
                // level's rows share a few runs of threads, and a cache line
                // of an ELL slot mostly serves rows that all occupy it
                const int mc = (slen[t] + 7) / 8;
                int p = 0;
                for (int q = 0; q < nrows; ++q) {
                    const int qc = (slen[q] + 7) / 8;
                    p += qc > mc || (qc == mc && (slev[q] < mine || (slev[q] == mine && q < t))) ? 1 : 0;
                }
                const int first = dir == 0 ? a : e;  // lowest row of the chunk
                perm[first + p] = make_int2(i, rlen);
                pos[i] = p;
            }
            __syncthreads();
        }
    }
}
void launch_bj_levels(int nblocks, const int* bp, const int* lrp, const int* lci, const int* urp, const int* uci,
                      const int2* lch, const int2* uch, int* llev, int* ulev, int* lnl, int* unl, int2* lperm,
                      int2* uperm, int* lpos, int* upos, hipStream_t s) {
    if (nblocks > 0)
        k_bj_levels<<<nblocks, kBjThreads, 0, s>>>(bp, lrp, lci, urp, uci, lch, uch, llev, ulev, lnl, unl, lperm,
                                                   uperm, lpos, upos);
}

// Chunk-interleaved copy of the newest kEll entries of every row of one
// triangle, right-aligned: slot u of the row at position t of its chunk
// [ca, cb) (t = pos[row], the thread that solves it) sits at
// ca * kEll + u * (cb - ca) + t (the chunk's slab is [ca, cb) * kEll) and
// holds the row's entry kEll - u from its end, so slot kEll - 1 is the
// entry nearest the diagonal; in FP64 and rounded to FP32.  Empty slots
// (below kEll - row length) hold a column no sweep takes before the row's
// level (forward: the row itself; backward: the row itself) and weight 0.
__global__ __launch_bounds__(256) void k_bj_ell(const int* __restrict__ bp, const int* __restrict__ rp,
                                                const int* __restrict__ ci, const double* __restrict__ val,
                                                const int* __restrict__ pos, int fwd, int* __restrict__ ec,
                                                double* __restrict__ ev64, float* __restrict__ ev32) {
    const int b = blockIdx.x;
    const int lo = bp[b], hi = bp[b + 1];
    for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) {
        int ca, cb;
        if (fwd)
            bj_chunk<true>(lo, hi, (i - lo) / kBjThreads, ca, cb);
        else
            bj_chunk<false>(lo, hi, (hi - 1 - i) / kBjThreads, ca, cb);
        const int nrows = cb - ca;
        const int r1 = rp[i + 1];
        const int nh = min(r1 - rp[i], kEll);
        const int64_t base = (int64_t)ca * kEll + pos[i];
        for (int u = 0; u < kEll - nh; ++u) {
            const int64_t at = base + (int64_t)u * nrows;
            ec[at] = i;
            ev64[at] = 0.0;
            ev32[at] = 0.0f;
        }
        for (int u = kEll - nh; u < kEll; ++u) {
            const int64_t at = base + (int64_t)u * nrows;
            const int e = r1 - kEll + u;
            const double w = val[e];
            ec[at] = ci[e];
            ev64[at] = w;
            ev32[at] = (float)w;
        }
    }
}
void launch_bj_ell(int nblocks, const int* bp, const int* rp, const int* ci, const double* val, const int* pos,
                   bool fwd, int* ec, double* ev64, float* ev32, hipStream_t s) {
    if (nblocks > 0) k_bj_ell<<<nblocks, 256, 0, s>>>(bp, rp, ci, val, pos, fwd ? 1 : 0, ec, ev64, ev32);
}

// Count and copy of the older entries of every row of one triangle (all
// but the newest kEll, in stored order) into a CSR of their own (orp, oci,
// ov64/ov32), so that the older entries of a chunk's rows are one
// contiguous range.
__global__ __launch_bounds__(256) void k_bj_old_count(int n, const int* __restrict__ rp, int* __restrict__ cnt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) cnt[i] = max(0, rp[i + 1] - rp[i] - kEll);
}
__global__ __launch_bounds__(256) void k_bj_old_copy(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ val, const int* __restrict__ orp,
                                                     int* __restrict__ oci, double* __restrict__ ov64,
                                                     float* __restrict__ ov32) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int r0 = rp[i], o0 = orp[i], no = orp[i + 1] - o0;
    for (int k = 0; k < no; ++k) {
        oci[o0 + k] = ci[r0 + k];
        ov64[o0 + k] = val[r0 + k];
        ov32[o0 + k] = (float)val[r0 + k];
    }
}
void launch_bj_old(int n, const int* rp, const int* ci, const double* val, int* cnt, int* tmp, int* orp, int* oci,
                   double* ov64, float* ov32, hipStream_t s) {
    const int g = (n + 255) / 256;
    if (n > 0) k_bj_old_count<<<g, 256, 0, s>>>(n, rp, cnt);
    launch_scan(n, cnt, orp, tmp, s);
    if (n > 0) k_bj_old_copy<<<g, 256, 0, s>>>(n, rp, ci, val, orp, oci, ov64, ov32);
}

// What a thread holds of its row in a chunk, loaded one chunk ahead.
template <typename V, typename F>
struct BjRow {
    int ec[kEll];  // newest entries (ELL copy, right-aligned)
    F ev[kEll];
    int len;       // entries in the row
    int o0;        // first older entry (older CSR)
    int obase;     // first older entry of the chunk
    int ocnt;      // older entries of the chunk
    V ar;          // r_i (forward), converted only when the chunk starts
    F a0;          // y_i (backward)
    F dg;          // u_ii (backward)
    V rr;          // r_i for (r, z) (backward, MODE 1/2)
    int lev;       // level inside the chunk
    int i;         // the row
};

// {row, entries} solved by thread t in chunk m (any row of the chunk for a
// thread past its end).
template <bool FWD>
__device__ __forceinline__ int2 bj_row(const BJDev& P, int lo, int hi, int m, int t) {
    int ca, cb;
    bj_chunk<FWD>(lo, hi, m, ca, cb);
    return (FWD ? P.lperm : P.uperm)[ca + min(t, cb - ca - 1)];
}

// Issue the loads of thread t's row il = {i, entries} of chunk m; only the
// occupied ELL slots are read.  orng = the chunk's older entries [first, end),
// read earlier.
template <bool FWD, int MODE, typename V, typename F>
__device__ __forceinline__ void bj_load(BjRow<V, F>& R, const BJDev& P, const V* rin, const F* y, int lo, int hi,
                                        int m, int t, int2 il, int2 orng) {
    int ca, cb;
    bj_chunk<FWD>(lo, hi, m, ca, cb);
    const int nrows = cb - ca;
    const int i = il.x;
    R.i = i;
    const int* __restrict__ orp = FWD ? P.lorp : P.uorp;
    const int* __restrict__ ec = FWD ? P.lell_c : P.uell_c;
    const F* __restrict__ ev = (const F*)(FWD ? P.lell_v : P.uell_v);
    R.obase = orng.x;
    R.ocnt = orng.y - orng.x;
    if (t < nrows) {
        R.len = il.y;
        R.o0 = orp[i];
        const unsigned base = (unsigned)ca * kEll + t;  // the copies hold fewer than 2^31 entries
        const int first = kEll - min(il.y, kEll);
#pragma unroll
        for (int u = 0; u < kEll; ++u) {
            if (u >= first) {
                R.ec[u] = ec[base + (unsigned)(u * nrows)];
                R.ev[u] = ev[base + (unsigned)(u * nrows)];
            } else {
                R.ec[u] = i;  // empty slot: the row itself, weight 0
                R.ev[u] = F(0);
            }
        }
        R.lev = FWD ? P.llev[i] : P.ulev[i];
        if (FWD) {
            R.ar = rin[i];
        } else {
            R.a0 = y[i];
            R.dg = ((const F*)P.udiag)[i];
            if (MODE == 1 || MODE == 2) R.rr = rin[i];
        }
    } else {
        R.len = 0;
        R.o0 = 0;
        R.lev = -1;
    }
}

// Solution value of row j from the ring or, when it has left the ring,
// from memory (forward: y; backward: z).
template <bool FWD, int RING, typename V, typename F, typename Bits>
__device__ __forceinline__ F bj_value(int j, bool inring, const Bits* ring, int lo, const F* y, const V* z) {
    if (inring) return from_bits<F>(lload(ring + ((j - lo) & (RING - 1))));
    return FWD ? gload(y + j) : (F)gload(z + j);
}

template <bool FWD, int MODE, typename V, typename F>
__device__ __forceinline__ void bj_sweep(const BJDev& P, const V* rin, F* y, V* z, int lo, int hi, int t,
                                         typename Sentinel<F>::Bits* ring, int* pka, F* pkw, int* soc, F* sov,
                                         F* spr, const int* nlg, double& rz, int& bad) {
    using Bits = typename Sentinel<F>::Bits;
    constexpr Bits SENT = Sentinel<F>::bits;
    constexpr int RING = BjRing<F>::size;
    constexpr unsigned ZOFF = RING * sizeof(Bits);  // byte offset of the ring's zero slot
    const int nch = (hi - lo + kBjThreads - 1) / kBjThreads;
    const int* __restrict__ oci = FWD ? P.loci : P.uoci;
    const F* __restrict__ oval = (const F*)(FWD ? P.lov : P.uov);
    const int* __restrict__ oorp = FWD ? P.lorp : P.uorp;
    const char* rbase = (const char*)ring;
    auto rd = [&](unsigned off) { return from_bits<F>(*(const Bits*)(rbase + off)); };
    BjRow<V, F> nx, cu;
    int sc[kStageOld / kBjThreads];
    F sv[kStageOld / kBjThreads];
    // the older-entry range of chunk m: {orp[first row], orp[end row]}
    auto orange = [&](int m) {
        int ca, cb;
        bj_chunk<FWD>(lo, hi, m, ca, cb);
        return make_int2(gload(oorp + ca), gload(oorp + cb));
    };
    // row indices run one chunk ahead of the row loads, and the older-entry
    // ranges two chunks ahead, so that the stage of the next chunk's older
    // entries never waits for that chunk's row loads
    bj_load<FWD, MODE>(nx, P, rin, y, lo, hi, 0, t, bj_row<FWD>(P, lo, hi, 0, t), orange(0));
    int2 orng1 = orange(min(1, nch - 1));
    // levels of chunk m, read a chunk ahead
    auto levels_of = [&](int m) { return gload(nlg + m); };
    int cnl1 = levels_of(0);
    int2 inext = bj_row<FWD>(P, lo, hi, min(1, nch - 1), t);
    auto stage_load = [&]() {
#pragma unroll
        for (int k = 0; k < kStageOld / kBjThreads; ++k) {
            const int e = t + k * kBjThreads;
            if (e < nx.ocnt) {
                sc[k] = oci[nx.obase + e];
                sv[k] = oval[nx.obase + e];
            }
        }
    };
    stage_load();
    for (int m = 0; m < nch; ++m) {
        cu = nx;
        int ca, cb;
        bj_chunk<FWD>(lo, hi, m, ca, cb);
        const int cnl = cnl1;
        const bool live = t < cb - ca;
        const int i = cu.i;
        // rows whose values are in the ring: forward [cb - RING, cb),
        // backward [ca, ca + RING); earlier chunks: forward j < ca,
        // backward j >= cb
        const int ring_edge = FWD ? cb - RING : ca + RING;
        const bool all_ring = FWD ? ring_edge <= lo : ring_edge >= hi;
        auto in_ring = [&](int j) { return FWD ? j >= ring_edge : j < ring_edge; };
        auto earlier = [&](int j) { return FWD ? j < ca : j >= cb; };
        auto roff = [&](int j) { return (unsigned)((j - lo) & (RING - 1)) * (unsigned)sizeof(Bits); };
        // the chunk's older entries go to LDS; for one on an earlier chunk
        // (its solution value is final) the thread staging it also forms its
        // product, so that the rows only subtract
        if (cu.ocnt > 0) {
#pragma unroll
            for (int k = 0; k < kStageOld / kBjThreads; ++k) {
                const int e = t + k * kBjThreads;
                if (e < cu.ocnt) {
                    soc[e] = sc[k];
                    sov[e] = sv[k];
                    spr[e] = earlier(sc[k]) ? sv[k] * bj_value<FWD, RING, V, F>(sc[k], in_ring(sc[k]), ring, lo, y, z)
                                            : F(0);
                }
            }
        }
        if (live) ring[(i - lo) & (RING - 1)] = SENT;
        __syncthreads();
        const F a0 = FWD ? (F)cu.ar : cu.a0;
        F acc = a0;
        const int nold = max(0, cu.len - kEll);
        const int first = kEll - min(cu.len, kEll);  // first occupied ELL slot
        int opos = 0;                                 // older entries taken
        int next = first;                             // first ELL slot not yet taken
        // older entry k of this row: staged in LDS, or from memory past the stage
        auto old_at = [&](int k, int& j, F& w) {
            const int s = cu.o0 - cu.obase + k;
            if (s < kStageOld) {
                j = lload(soc + s);
                w = lload(sov + s);
            } else {
                j = gload(oci + cu.o0 + k);
                w = gload(oval + cu.o0 + k);
            }
        };
        if (live) {
            // older entries while on earlier chunks: the staged ones as
            // ready products, four at a time; any past the stage through the
            // general path
            bool open = true;
            const int sb = cu.o0 - cu.obase;
            while (open && opos < nold && sb + opos < kStageOld) {
                int jj[4];
                F pp[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (opos + u < nold && sb + opos + u < kStageOld) {
                        jj[u] = soc[sb + opos + u];
                        pp[u] = spr[sb + opos + u];
                    }
                }
                const int o4 = opos;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (open && o4 + u < nold && sb + o4 + u < kStageOld) {
                        if (earlier(jj[u])) {
                            acc = acc - pp[u];
                            ++opos;
                        } else {
                            open = false;
                        }
                    }
                }
            }
            while (open && opos < nold) {
                int jj[4];
                F ww[4], vv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (opos + u < nold) old_at(opos + u, jj[u], ww[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (opos + u < nold && earlier(jj[u]))
                        vv[u] = bj_value<FWD, RING, V, F>(jj[u], in_ring(jj[u]), ring, lo, y, z);
                const int o4 = opos;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (open && o4 + u < nold) {
                        if (earlier(jj[u])) {
                            acc = acc - ww[u] * vv[u];
                            ++opos;
                        } else {
                            open = false;
                        }
                    }
                }
            }
            if (opos == nold) {
                // ELL slots on earlier chunks: a prefix, by the sort order
                // (empty slots hold the row itself, never earlier).  Slots
                // not taken read the zero slot; their weights are finite.
                if (all_ring) {
#pragma unroll
                    for (int u = 0; u < kEll; ++u) {
                        const bool tk = earlier(cu.ec[u]);
                        acc = acc - cu.ev[u] * rd(tk ? roff(cu.ec[u]) : ZOFF);
                        next = tk ? u + 1 : next;
                    }
                } else {
                    // four slots at a time: their values first (the reads
                    // in flight together), then the terms in slot order
#pragma unroll
                    for (int u0 = 0; u0 < kEll; u0 += 4) {
                        F vv[4];
#pragma unroll
                        for (int u = u0; u < u0 + 4; ++u) {
                            vv[u - u0] = F(0);
                            if (u >= first && earlier(cu.ec[u]))
                                vv[u - u0] = bj_value<FWD, RING, V, F>(cu.ec[u], in_ring(cu.ec[u]), ring, lo, y, z);
                        }
#pragma unroll
                        for (int u = u0; u < u0 + 4; ++u) {
                            if (u >= first && earlier(cu.ec[u])) {
                                acc = acc - cu.ev[u] * vv[u - u0];
                                next = u + 1;
                            }
                        }
                    }
                }
            }
        }
        // what is left is on this chunk (the entries are sorted), so in the
        // ring at the row's level: the newest kHeld slots stay in registers
        // as (ring offset, weight), the others are parked in this thread's
        // LDS list, padded to a multiple of four with zero terms
        unsigned hoff[kHeld];
        F hw[kHeld];
#pragma unroll
        for (int h = 0; h < kHeld; ++h) {
            const int u = kPark + h;
            const bool keep = live && u >= next;
            hoff[h] = keep ? roff(cu.ec[u]) : ZOFF;
            hw[h] = cu.ev[u];  // finite; a slot not kept reads the zero slot
        }
        const int npark = live ? max(0, kPark - next) : 0;
#pragma unroll
        for (int u = 0; u < kPark; ++u) {
            if (live && u >= next) {
                pka[(u - next) * kBjThreads + t] = (int)roff(cu.ec[u]);
                pkw[(u - next) * kBjThreads + t] = cu.ev[u];
            }
        }
        const int npad = (npark + 3) & ~3;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (npark + q < npad) {
                pka[(npark + q) * kBjThreads + t] = (int)ZOFF;
                pkw[(npark + q) * kBjThreads + t] = F(0);
            }
        }
        // the next chunk's rows load while this one is solved (not hoisted
        // above the straight pass, whose registers they would otherwise
        // share); the last chunk loads itself again, so that the loads, and
        // the registers they fill, are unconditional
        __builtin_amdgcn_sched_barrier(0);
        bj_load<FWD, MODE>(nx, P, rin, y, lo, hi, min(m + 1, nch - 1), t, inext, orng1);
        inext = bj_row<FWD>(P, lo, hi, min(m + 2, nch - 1), t);
        auto level = [&](int lv) {
            if (live && cu.lev == lv) {
                // older entries left (only when an older entry is on this
                // chunk): the staged ones, then any past the stage, in two
                // loops so that waiting for a load from memory never also
                // waits for the staged path (and the next chunk's loads)
                auto older = [&](int j, F w) {
                    const Bits vb = ring[(j - lo) & (RING - 1)];
                    bad |= vb == SENT;
                    acc = acc - w * from_bits<F>(vb);
                };
                const int sb = cu.o0 - cu.obase;
                for (; opos < nold && sb + opos < kStageOld; ++opos)
                    older(lload(soc + sb + opos), lload(sov + sb + opos));
                for (; opos < nold; ++opos) older(gload(oci + cu.o0 + opos), gload(oval + cu.o0 + opos));
                for (int k = 0; k < npad; k += 4) {
                    unsigned oo[4];
                    F ww[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        oo[u] = (unsigned)pka[(k + u) * kBjThreads + t];
                        ww[u] = pkw[(k + u) * kBjThreads + t];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = acc - ww[u] * rd(oo[u]);
                }
#pragma unroll
                for (int h = 0; h < kHeld; ++h) acc = acc - hw[h] * rd(hoff[h]);
                const F out = FWD ? acc : acc / cu.dg;
                // a sentinel read turns the row into NaN
                bad |= (out != out) && (a0 == a0);
                ring[(i - lo) & (RING - 1)] = to_bits<F>(out);
                if (FWD) {
                    y[i] = out;
                } else {
                    const V zv = (V)out;
                    z[i] = zv;
                    if (MODE == 1 || MODE == 2) rz += (double)cu.rr * (double)zv;
                }
            }
            __syncthreads();
        };
        // the next chunk's older entries load with its rows (their range
        // was read a chunk earlier), and the range of the chunk after it
        // last (waited for at the end of this chunk, with the row loads)
        stage_load();
        const int2 orng2 = orange(min(m + 2, nch - 1));
        const int cnl2 = levels_of(min(m + 1, nch - 1));
        for (int lv = 0; lv < cnl; ++lv) level(lv);
        orng1 = orng2;
        cnl1 = cnl2;
    }
}

template <typename V, typename F, int MODE>
__device__ __forceinline__ void bj_body(const BJDev& P, const PcgVecs& Vv, KrylovState* st, int it, int bid) {
    using Bits = typename Sentinel<F>::Bits;
    constexpr int RING = BjRing<F>::size;
    __shared__ Bits ring[RING + 1];
    __shared__ int pka[kPark * kBjThreads];
    __shared__ F pkw[kPark * kBjThreads];
    __shared__ int soc[kStageOld];
    __shared__ F sov[kStageOld];
    __shared__ F spr[kStageOld];
    __shared__ double red[16];
    __shared__ int shd;
    const int b = bid, t = threadIdx.x;
    const int nb = P.nblocks;
    const int lo = P.bp[b], hi = P.bp[b + 1];
    if (t == 0) ring[RING] = to_bits<F>(F(0));
    __syncthreads();
    V* __restrict__ z = (V*)Vv.z;
    F* __restrict__ y = (F*)Vv.y;
    V* r = (V*)Vv.r;

    if (MODE == 0 && st && block_done(st, &shd)) return;
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
        // four rows per thread in flight; each thread adds its rows in order
        for (int i0 = lo + t; i0 < hi; i0 += 4 * kBjThreads) {
            V pv[4], qv[4], xv[4], rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * kBjThreads;
                if (i < hi) {
                    pv[u] = p[i];
                    qv[u] = q[i];
                    xv[u] = x[i];
                    rv[u] = r[i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * kBjThreads;
                if (i < hi) {
                    x[i] = xv[u] + a * pv[u];
                    const V ri = rv[u] - a * qv[u];
                    r[i] = ri;
                    rr += (double)ri * (double)ri;
                }
            }
        }
        rr = block_sum(rr, red);  // also orders the r updates before the sweeps read them
        if (t == 0) Vv.part_rr[b] = rr;
    }
    int bad = 0;
    double rz = 0.0;
    // forward substitution y_i = r_i - sum_{j<i} l_ij y_j (MODE 4: y given)
    if (MODE != 4 && lo < hi) bj_sweep<true, MODE, V, F>(P, r, y, z, lo, hi, t, ring, pka, pkw, soc, sov, spr, P.lnl + lo + b, rz, bad);
    // backward substitution z_i = (y_i - sum_{j>i} u_ij z_j) / u_ii (MODE 3: not done)
    if (MODE != 3 && lo < hi) bj_sweep<false, MODE, V, F>(P, r, y, z, lo, hi, t, ring, pka, pkw, soc, sov, spr, P.unl + lo + b, rz, bad);
    if (bad && st) atomicExch(&st->spin_err, 1);
    if (MODE == 1 || MODE == 2) {
        rz = block_sum(rz, red);
        if (t == 0) Vv.part_rz[(it & 1) * nb + b] = rz;
    }
}
template <typename V, typename F, int MODE>
__global__ __launch_bounds__(kBjThreads) void k_bj(BJDev P, PcgVecs Vv, KrylovState* st, int it) {
    bj_body<V, F, MODE>(P, Vv, st, it, blockIdx.x);
}


template <typename V, typename F>
void launch_bj(int mode, const BJDev& P, const PcgVecs& v, KrylovState* st, int it, hipStream_t s) {
    if (P.nblocks <= 0) return;
    switch (mode) {
        case 0: k_bj<V, F, 0><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it); break;
        case 1: k_bj<V, F, 1><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it); break;
        case 2: k_bj<V, F, 2><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it); break;
        case 3: k_bj<V, F, 3><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it); break;
        default: k_bj<V, F, 4><<<P.nblocks, kBjThreads, 0, s>>>(P, v, st, it); break;
    }
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
// The border's t = U^T z and s = K^{-1} t from the projection's slice
// partials (each column's slices added in slice order, then K^{-1} t row by
// row), into the shared arrays ts and ss; every workgroup of the consumer
// folds for itself.  Reached by all threads of the workgroup.
__device__ __forceinline__ void border_fold(const BorderDev& bd, double* ts, double* ss) {
    const int k = bd.k, sl = bd.slices;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double t = 0.0;
        for (int q = 0; q < sl; ++q) t += bd.part[j * sl + q];
        ts[j] = t;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double t = 0.0;
        for (int i = 0; i < k; ++i) t = fma(bd.Kinv[j * k + i], ts[i], t);
        ss[j] = t;
    }
    __syncthreads();
}

template <typename T, bool BORDER>
__device__ __forceinline__ void pupdate_body(int n, T* __restrict__ p, const T* __restrict__ z,
                                             const double* __restrict__ part_rz, const double* __restrict__ part_rr,
                                             int nb, const BorderDev& bd, KrylovState* st, int it, int mode, int bid,
                                             int gdim) {
    __shared__ double red[8];
    __shared__ double ts[64];
    __shared__ double ss[64];
    __shared__ double fp[kMaxRank * 32];
    __shared__ int shd;
    // The loads the workgroup needs are issued before any of them is used,
    // so that their latencies overlap instead of adding up: the (r,r) and
    // (r,z) partials, the border's slice partials and rows of K^{-1}, and
    // this thread's first row (z, p and its border columns).  The
    // arithmetic and its order are those of the plain sequence.
    constexpr int kPre = 24;  // border columns held in registers
    constexpr int kPart = 8;  // staged values (slice partials, then K^{-1}) per thread
    const int t = threadIdx.x;
    const int g = gdim;
    const int per = (n + g - 1) / g;
    const int r0 = bid * per, r1 = min(n, r0 + per);
    const int i0 = r0 + t;
    const bool has0 = i0 < r1;
    const T z0 = has0 ? z[i0] : T(0);
    const T p0 = has0 && mode != PUPD_START ? p[i0] : T(0);
    const bool one = nb <= (int)blockDim.x;  // at most one partial per thread
    const double prr = one && mode == PUPD_STEP && t < nb ? part_rr[t] : 0.0;
    const double prz = one && t < nb ? part_rz[(it & 1) * nb + t] : 0.0;
    const int k = BORDER ? bd.k : 0;
    const int m = BORDER ? k * bd.slices : 0;  // slice partials; K^{-1} follows them in fp
    const int mk = m + k * k;
    const bool pre = BORDER && k <= kPre;
    const bool stage = BORDER && mk <= kPart * (int)blockDim.x && mk <= kMaxRank * 32;
    double wv[kPre], pv[kPart];
    if (BORDER) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) wv[u] = pre && has0 && u < k ? bd.W[(size_t)u * n + i0] : 0.0;
#pragma unroll
        for (int u = 0; u < kPart; ++u) {
            const int q = t + u * (int)blockDim.x;
            pv[u] = !stage || q >= mk ? 0.0 : (q < m ? bd.part[q] : bd.Kinv[q - m]);
        }
    }
    auto sum_partials = [&](const double* a, double mine) {
        if (!one) return block_sum_array(a, nb, red);
        double s = 0.0;
        if (t < nb) s += mine;
        return block_sum(s, red);
    };
    if (mode == PUPD_STEP) {
        if (block_done(st, &shd)) return;
        const double rr = sum_partials(part_rr, prr);
        const bool conv = rr <= st->tol2 * st->bb;
        const bool upd = rr < st->delta2 * st->rr0 ||
                         (st->refine_every > 0 && it + 1 - st->it_refine >= st->refine_every);
        if (conv || upd) {
            if (bid == 0 && t == 0) {
                st->conv = conv ? 1 : 0;
                st->update = upd ? 1 : 0;
                st->iters = it + 1;
                set_done(st);
            }
            return;
        }
    }
    double rz = sum_partials(part_rz + (it & 1) * nb, prz);
    if (BORDER) {
        if (stage) {
            // t = U^T z and s = K^{-1} t as border_fold computes them
#pragma unroll
            for (int u = 0; u < kPart; ++u) {
                const int q = t + u * (int)blockDim.x;
                if (q < mk) fp[q] = pv[u];
            }
            __syncthreads();
            const int sl = bd.slices;
            if (t < k) {
                double a = 0.0;
                for (int q = 0; q < sl; ++q) a += fp[t * sl + q];
                ts[t] = a;
            }
            __syncthreads();
            if (t < k) {
                double a = 0.0;
                for (int i = 0; i < k; ++i) a = fma(fp[m + t * k + i], ts[i], a);
                ss[t] = a;
            }
            __syncthreads();
        } else {
            border_fold(bd, ts, ss);
        }
        double ts_dot = 0.0;
        for (int j = 0; j < k; ++j) ts_dot = fma(ts[j], ss[j], ts_dot);
        rz -= ts_dot;
    }
    double beta = 0.0;
    if (mode != PUPD_START) beta = rz / st->rzs[(it + 1) & 1];
    if (!isfinite(beta) || !isfinite(rz)) {
        if (bid == 0 && t == 0) {
            st->breakdown = 1;
            st->iters = it + 1;
            set_done(st);
        }
        return;
    }
    if (BORDER && bd.up && bid == 0) {
        // the next product's low-rank coefficients: U^T p = t - G s + beta U^T p_old
        for (int j = t; j < bd.k; j += blockDim.x) {
            double u = ts[j];
            for (int i = 0; i < bd.k; ++i) u = fma(-bd.G[j * bd.k + i], ss[i], u);
            if (mode != PUPD_START) u = fma(beta, bd.up[j], u);
            bd.up[j] = u;
            bd.ufold[j] = bd.c[j] * u;
        }
    }
    const T bt = (T)beta;
    const double* W = bd.W;
    for (int i = i0; i < r1; i += blockDim.x) {
        const bool first = i == i0;
        T zi = first ? z0 : z[i];
        if (BORDER) {
            double c = 0.0;
            if (pre && first) {
#pragma unroll
                for (int j = 0; j < kPre; ++j)
                    if (j < k) c = fma(wv[j], ss[j], c);
            } else {
                for (int j = 0; j < k; ++j) c = fma(W[(size_t)j * n + i], ss[j], c);
            }
            zi = (T)((double)zi - c);
        }
        p[i] = (mode == PUPD_START) ? zi : zi + bt * (first ? p0 : p[i]);
    }
    if (bid == 0 && t == 0) st->rzs[it & 1] = rz;
}
template <typename T, bool BORDER>
__global__ __launch_bounds__(256) void k_pcg_pupdate(int n, T* __restrict__ p, const T* __restrict__ z,
                                                     const double* __restrict__ part_rz,
                                                     const double* __restrict__ part_rr, int nb, BorderDev bd,
                                                     KrylovState* st, int it, int mode) {
    pupdate_body<T, BORDER>(n, p, z, part_rz, part_rr, nb, bd, st, it, mode, blockIdx.x, gridDim.x);
}


// one row per thread (every workgroup resident at once up to ~1M rows)
int pupdate_grid(int n) {
    int g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    return g < 1 ? 1 : g;
}

template <typename T>
void launch_pcg_pupdate(int n, const PcgVecs& v, int nblocks, const BorderDev& bd, KrylovState* st, int it,
                        int mode, hipStream_t s) {
    const int g = pupdate_grid(n);
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

// ------------------------------------------------------------------ shared launches
// The slot that owns workgroup w (slots in launch order; ns is small, and
// the table sits in the scalar cache after the first workgroups).
__device__ __forceinline__ int slot_of(const int* __restrict__ pre, int ns, int w) {
    int s = 0;
    while (s + 1 < ns && pre[s + 1] <= w) ++s;
    return s;
}

template <typename V, typename F, int G>
__global__ __launch_bounds__(kSpmvThreads) void k_spmv_slots(const int* __restrict__ pre,
                                                             const SpmvSlot* __restrict__ tab, int ns) {
    const int s = slot_of(pre, ns, blockIdx.x);
    const SpmvSlot d = tab[s];
    const int w = blockIdx.x - pre[s];
    if (w >= d.grid) return;  // padding to the next multiple of 8
    const LowRankDev none{};
    spmv_body<V, F, G, 4, false>(d.n, d.rp, d.ci, (const F*)d.v, (const V*)d.x, (V*)d.y, d.part_dot, d.st, none,
                                 d.halo, d.rows, w, d.grid);
}

template <typename V, typename F>
__global__ __launch_bounds__(kBjThreads) void k_bj_slots(const int* __restrict__ pre, const BjSlot* __restrict__ tab,
                                                         int ns, int k) {
    const int s = slot_of(pre, ns, blockIdx.x);
    const int w = blockIdx.x - pre[s];
    const BjSlot& d = tab[s];
    if (w >= d.P.nblocks) return;
    bj_body<V, F, 1>(d.P, d.Vv, d.st, d.it0 + k, w);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pupdate_slots(const int* __restrict__ pre, const PupdSlot* __restrict__ tab,
                                                       int ns, int k) {
    const int s = slot_of(pre, ns, blockIdx.x);
    const PupdSlot d = tab[s];
    const int w = blockIdx.x - pre[s];
    if (w >= d.grid) return;
    const BorderDev none{};
    pupdate_body<T, false>(d.n, (T*)d.p, (const T*)d.z, d.part_rz, d.part_rr, d.nb, none, d.st, d.it0 + k,
                           PUPD_STEP, w, d.grid);
}

template <typename V, typename F>
void launch_slots_iteration(const SlotTable& t, int ns, int k, int lanes, const int* wg, size_t shm,
                            hipStream_t s) {
    if (ns <= 0) return;
    constexpr int T = kSpmvThreads;
    switch (lanes) {
        case 64: k_spmv_slots<V, F, 64><<<wg[0], T, shm, s>>>(t.spmv_pre, t.spmv, ns); break;
        case 32: k_spmv_slots<V, F, 32><<<wg[0], T, shm, s>>>(t.spmv_pre, t.spmv, ns); break;
        case 16: k_spmv_slots<V, F, 16><<<wg[0], T, shm, s>>>(t.spmv_pre, t.spmv, ns); break;
        case 8: k_spmv_slots<V, F, 8><<<wg[0], T, shm, s>>>(t.spmv_pre, t.spmv, ns); break;
        default: k_spmv_slots<V, F, 4><<<wg[0], T, shm, s>>>(t.spmv_pre, t.spmv, ns); break;
    }
    k_bj_slots<V, F><<<wg[1], kBjThreads, 0, s>>>(t.bj_pre, t.bj, ns, k);
    k_pupdate_slots<V><<<wg[2], 256, 0, s>>>(t.pu_pre, t.pu, ns, k);
}
template void launch_slots_iteration<double, double>(const SlotTable&, int, int, int, const int*, size_t,
                                                     hipStream_t);
template void launch_slots_iteration<double, float>(const SlotTable&, int, int, int, const int*, size_t,
                                                    hipStream_t);
template void launch_slots_iteration<float, float>(const SlotTable&, int, int, int, const int*, size_t,
                                                   hipStream_t);

// ------------------------------------------------------------------ BiCGSTAB
// Vector steps of right-preconditioned BiCGSTAB (van der Vorst 1992; the
// paper's block-Jacobi solver, Sec. 4.3) with every scalar on the device:
// each workgroup sums, in the same fixed order, the partials it needs, so no
// scalar goes through the host.  The products and preconditioner applies
// between the steps are the SpMV and block-Jacobi launches.  The scalars of
// iteration `it` live at parity it & 1 (those of it - 1 at the other one);
// every kernel is a no-op once the state says done.
constexpr int kBicgThreads = 256;
int bicg_grid(int n) {
    int g = (n + kBicgThreads - 1) / kBicgThreads;
    return g < 1 ? 1 : (g > 4096 ? 4096 : g);
}

// pa[w] = workgroup w's share of (a, b); with c, pc[w] of (c, d)
__global__ __launch_bounds__(kBicgThreads) void k_dot2(int n, const double* __restrict__ a,
                                                       const double* __restrict__ b, const double* __restrict__ c,
                                                       const double* __restrict__ d, double* __restrict__ pa,
                                                       double* __restrict__ pc, const KrylovState* st) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const int g = gridDim.x, per = (n + g - 1) / g;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double s1 = 0.0, s2 = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        s1 = fma(a[i], b[i], s1);
        if (c) s2 = fma(c[i], d[i], s2);
    }
    s1 = block_sum(s1, red);
    if (c) s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        pa[blockIdx.x] = s1;
        if (c) pc[blockIdx.x] = s2;
    }
}
void launch_dot2(int n, const double* a, const double* b, const double* c, const double* d, double* pa, double* pc,
                 const KrylovState* st, hipStream_t s) {
    k_dot2<<<bicg_grid(n), kBicgThreads, 0, s>>>(n, a, b, c, d, pa, pc, st);
}

__device__ __forceinline__ void bicg_stop(KrylovState* st, int iters, int conv) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->conv = conv;
        st->breakdown = conv ? 0 : 1;
        st->iters = iters;
        set_done(st);
    }
}

// Start of iteration it: the residual of it - 1 meets the tolerance ->
// converged (iters = it); rho = (r^, r); p = r (first step of a cycle) or
// p = r + beta (p - omega v), beta = (rho / rho_prev)(alpha / omega).
__global__ __launch_bounds__(kBicgThreads) void k_bicg_p(int n, const double* __restrict__ r, double* __restrict__ p,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ part_rho,
                                                         const double* __restrict__ part_rr, KrylovState* st, int it,
                                                         int first) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const int m = gridDim.x;
    const double rho = block_sum_array(part_rho, m, red);
    if (!first) {
        const double rr = block_sum_array(part_rr, m, red);
        if (rr <= st->tol2 * st->bb) { bicg_stop(st, it, 1); return; }
    }
    const int q = (it + 1) & 1;
    const double om = first ? 1.0 : st->bi_omega[q];
    const double beta = first ? 0.0 : (rho / st->bi_rho[q]) * (st->bi_alpha[q] / om);
    if (rho == 0.0 || !isfinite(rho) || !isfinite(beta) || om == 0.0) { bicg_stop(st, it, 0); return; }
    const int per = (n + m - 1) / m;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x)
        p[i] = first ? r[i] : r[i] + beta * (p[i] - om * v[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->bi_rho[it & 1] = rho;
}
void launch_bicg_p(int n, const double* r, double* p, const double* v, const double* part_rho, const double* part_rr,
                   KrylovState* st, int it, bool first, hipStream_t s) {
    k_bicg_p<<<bicg_grid(n), kBicgThreads, 0, s>>>(n, r, p, v, part_rho, part_rr, st, it, first ? 1 : 0);
}

// alpha = rho / (r^, v); s = r - alpha v; partials of ||s||^2
__global__ __launch_bounds__(kBicgThreads) void k_bicg_s(int n, const double* __restrict__ r,
                                                         const double* __restrict__ v, double* __restrict__ sv,
                                                         const double* __restrict__ part_rv,
                                                         double* __restrict__ part_ss, KrylovState* st, int it) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const int m = gridDim.x;
    const double rv = block_sum_array(part_rv, m, red);
    const double alpha = st->bi_rho[it & 1] / rv;
    if (rv == 0.0 || !isfinite(alpha)) { bicg_stop(st, it, 0); return; }
    const int per = (n + m - 1) / m;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double ss = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const double si = r[i] - alpha * v[i];
        sv[i] = si;
        ss = fma(si, si, ss);
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) part_ss[blockIdx.x] = ss;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->bi_alpha[it & 1] = alpha;
}
void launch_bicg_s(int n, const double* r, const double* v, double* sv, const double* part_rv, double* part_ss,
                   KrylovState* st, int it, hipStream_t s) {
    k_bicg_s<<<bicg_grid(n), kBicgThreads, 0, s>>>(n, r, v, sv, part_rv, part_ss, st, it);
}

// End of iteration it: if ||s|| meets the tolerance, x += alpha ph and
// r = s (converged, iters = it + 1); otherwise omega = (t, s) / (t, t),
// x += alpha ph + omega sh, r = s - omega t, and the partials of (r^, r) and
// ||r||^2 for the next iteration.
__global__ __launch_bounds__(kBicgThreads) void k_bicg_x(
    int n, double* __restrict__ x, const double* __restrict__ ph, const double* __restrict__ sh,
    const double* __restrict__ sv, const double* __restrict__ t, double* __restrict__ r, const double* __restrict__ rh,
    const double* __restrict__ part_ss, const double* __restrict__ part_ts, const double* __restrict__ part_tt,
    double* __restrict__ part_rho, double* __restrict__ part_rr, KrylovState* st, int it) {
    __shared__ double red[8];
    __shared__ int shd;
    if (block_done(st, &shd)) return;
    const int m = gridDim.x;
    const double ss = block_sum_array(part_ss, m, red);
    const double alpha = st->bi_alpha[it & 1];
    const int per = (n + m - 1) / m;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    if (ss <= st->tol2 * st->bb) {
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            x[i] = x[i] + alpha * ph[i];
            r[i] = sv[i];
        }
        bicg_stop(st, it + 1, 1);
        return;
    }
    const double ts = block_sum_array(part_ts, m, red);
    const double tt = block_sum_array(part_tt, m, red);
    const double omega = ts / tt;
    if (tt == 0.0 || !isfinite(omega)) { bicg_stop(st, it + 1, 0); return; }
    double rho = 0.0, rr = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        x[i] = x[i] + alpha * ph[i] + omega * sh[i];
        const double ri = sv[i] - omega * t[i];
        r[i] = ri;
        rho = fma(rh[i], ri, rho);
        rr = fma(ri, ri, rr);
    }
    rho = block_sum(rho, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        part_rho[blockIdx.x] = rho;
        part_rr[blockIdx.x] = rr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->bi_omega[it & 1] = omega;
}
void launch_bicg_x(int n, double* x, const double* ph, const double* sh, const double* sv, const double* t, double* r,
                   const double* rh, const double* part_ss, const double* part_ts, const double* part_tt,
                   double* part_rho, double* part_rr, KrylovState* st, int it, hipStream_t s) {
    k_bicg_x<<<bicg_grid(n), kBicgThreads, 0, s>>>(n, x, ph, sh, sv, t, r, rh, part_ss, part_ts, part_tt, part_rho,
                                                     part_rr, st, it);
}

// ------------------------------------------------------------------ GCR(m)
// End of a GCR step (right preconditioned, Sec. 2.2; Eisenstat, Elman and
// Schultz 1983): q = M p has been made orthogonal to the cycle's earlier
// directions, *nu2 = ||q||^2 after and *nu02 before the projections.  When
// nu2 > 1e-28 nu02 (else the direction adds nothing: a breakdown, nothing
// is written): q /= nu and p /= nu are stored, alpha = (r, q) / nu from the
// partials of (r, q) taken before the scaling, x += alpha p, r -= alpha q,
// and part_rr[w] = the workgroup's share of ||r||^2.
__global__ __launch_bounds__(kBicgThreads) void k_gcr_xr(int n, double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ p, double* __restrict__ q,
                                                         const double* __restrict__ nu2, const double* __restrict__ nu02,
                                                         const double* __restrict__ part_rq,
                                                         double* __restrict__ part_rr) {
    __shared__ double red[8];
    const int m = gridDim.x;
    const double v2 = nu2[0];
    const bool ok = v2 > 1e-28 * nu02[0] && isfinite(v2);
    const double inv = ok ? 1.0 / sqrt(v2) : 0.0;
    const double alpha = ok ? block_sum_array(part_rq, m, red) * inv : 0.0;
    const int per = (n + m - 1) / m;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double rr = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double ri = r[i];
        if (ok) {
            const double pi = p[i] * inv, qi = q[i] * inv;
            p[i] = pi;
            q[i] = qi;
            x[i] = x[i] + alpha * pi;
            ri = ri - alpha * qi;
            r[i] = ri;
        }
        rr = fma(ri, ri, rr);
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = rr;
}
void launch_gcr_xr(int n, double* x, double* r, double* p, double* q, const double* nu2, const double* nu02,
                   const double* part_rq, double* part_rr, hipStream_t s) {
    k_gcr_xr<<<bicg_grid(n), kBicgThreads, 0, s>>>(n, x, r, p, q, nu2, nu02, part_rq, part_rr);
}

// z <- z - W s, s = Kinv (sum of the U^T z partials): the border correction
// on its own (the solve loop fuses it into the direction update)
template <typename T>
__global__ __launch_bounds__(256) void k_border_fix(int n, T* __restrict__ z, BorderDev bd) {
    __shared__ double ts[kMaxRank];
    __shared__ double ss[kMaxRank];
    const int k = bd.k;
    border_fold(bd, ts, ss);
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
                                                  double* __restrict__ K, double* __restrict__ G) {
    __shared__ double red[8];
    const int a = blockIdx.x / k, b = blockIdx.x % k;
    double s = 0.0;
    for (int p = ucp[a] + threadIdx.x; p < ucp[a + 1]; p += blockDim.x) s = fma(ucv[p], W[(size_t)b * n + uri[p]], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        K[a * k + b] = s + (a == b ? 1.0 / c[a] : 0.0);
        G[a * k + b] = s;  // (U^T W)_ab
    }
}
void launch_border_k(int n, int k, const int* ucp, const int* uri, const double* ucv, const double* c,
                     const double* W, double* K, double* G, hipStream_t s) {
    k_border_k<<<k * k, 256, 0, s>>>(n, k, ucp, uri, ucv, c, W, K, G);
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
