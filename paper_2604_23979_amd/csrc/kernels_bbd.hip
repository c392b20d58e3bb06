// Bordered-block-diagonal (BBD) preconditioner kernels (paper Sec. 2.4):
// the dense Schur complement of the border, its LU factorisation with
// partial pivoting and explicit inverse on FP64 matrix cores, and the pieces
// of the Schur-coupled apply.
//
// Dense matrices are row-major FP64.  Per interior block b with tail
// [t_b, hi_b) (the rows/columns that couple to the border):
//   H_b  (t x ne, row-major) = L_TT^{-1} E_T[:, ecols_b]
//   Gt_b (t x nf, row-major) = (F_T[frows_b, :] U_TT^{-1})^T
//   S = C - sum_b scatter(Gt_b^T H_b)
#include "common.hpp"

namespace sdsl {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ GEMM
// C(map) -= A * B with A M x K (A_T: a[k * lda + i], else a[i * lda + k]),
// B K x N row-major, C row-major; rmap/cmap (nullable) send row i / column j
// of the product to C row rmap[i] / column cmap[j].  A 256-thread workgroup
// computes a 64 x 64 tile with v_mfma_f64_16x16x4f64: wave (wr, wc) owns the
// 32 x 32 quarter, 2 x 2 MFMA tiles, K staged through LDS 16 at a time.
// Operand layouts of the 16x16x4 FP64 MFMA: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; it receives D[l / 16 + 4 v][l % 16], v = 0..3.
constexpr int kGT = 64;   // tile edge
constexpr int kGK = 16;   // K per LDS stage

template <bool A_T>
__global__ __launch_bounds__(256) void k_dgemm_sub(int M, int N, int K, const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ B, int64_t ldb, double* C,
                                                   int64_t ldc, const int* __restrict__ rmap,
                                                   const int* __restrict__ cmap) {
    __shared__ double As[kGT][kGK + 1];
    __shared__ double Bs[kGK][kGT + 1];
    const int t = threadIdx.x;
    const int i0 = blockIdx.y * kGT, j0 = blockIdx.x * kGT;
    const int wave = t / kWave, lane = t % kWave;
    const int wr = (wave / 2) * 32, wc = (wave % 2) * 32;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += kGK) {
        // stage A (64 x 16) and B (16 x 64): 1024 values each, 4 per thread
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + u * 256;
            int ii, kk;
            if (A_T) { kk = e / kGT; ii = e % kGT; }   // contiguous along i
            else { ii = e / kGK; kk = e % kGK; }       // contiguous along k
            const int gi = i0 + ii, gk = k0 + kk;
            double av = 0.0;
            if (gi < M && gk < K) av = A_T ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
            As[ii][kk] = av;
            const int bk = e / kGT, bj = e % kGT;
            const int gbk = k0 + bk, gj = j0 + bj;
            Bs[bk][bj] = (gbk < K && gj < N) ? B[(int64_t)gbk * ldb + gj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            double af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[wr + a * 16 + lane % 16][ks + lane / 16];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[ks + lane / 16][wc + b * 16 + lane % 16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wr + a * 16 + lane / 16 + 4 * v;
                const int j = j0 + wc + b * 16 + lane % 16;
                if (i < M && j < N) {
                    const int64_t ci = rmap ? rmap[i] : i, cj = cmap ? cmap[j] : j;
                    C[ci * ldc + cj] -= acc[a][b][v];
                }
            }
}
void launch_dgemm_sub(bool a_t, int M, int N, int K, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double* C, int64_t ldc, const int* rmap, const int* cmap, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return;
    const dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
    if (a_t) k_dgemm_sub<true><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, rmap, cmap);
    else k_dgemm_sub<false><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, rmap, cmap);
}

// ------------------------------------------------------------------ LU
constexpr int kPanel = kLuPanel;  // panel width of the blocked LU

// Panel [k0, k0 + w) of the row-major n x n matrix S: for each column kk,
// the pivot is the first row of largest |S[i][kk]| (i >= kk), its row is
// swapped with row kk across all n columns, the column below is divided by
// the pivot and the panel's later columns get the rank-1 update.  One
// 1024-thread workgroup.  bad[0] is set when a pivot is zero.
__global__ __launch_bounds__(1024) void k_lu_panel(int n, int k0, int w, double* S, int* piv, int* bad) {
    __shared__ double bv[16];
    __shared__ int bi[16];
    __shared__ int sp;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int kk = k0; kk < k0 + w; ++kk) {
        double best = -1.0;
        int idx = n;
        for (int i = kk + t; i < n; i += nt) {
            const double a = fabs(S[(int64_t)i * n + kk]);
            if (a > best) { best = a; idx = i; }   // ascending i: first maximum kept
        }
        // wave then workgroup reduction: larger value, then smaller index
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_down(best, o, kWave);
            const int oi = __shfl_down(idx, o, kWave);
            if (ob > best || (ob == best && oi < idx)) { best = ob; idx = oi; }
        }
        if (t % kWave == 0) { bv[t / kWave] = best; bi[t / kWave] = idx; }
        __syncthreads();
        if (t == 0) {
            double b0 = bv[0];
            int i0 = bi[0];
            for (int q = 1; q < nt / kWave; ++q)
                if (bv[q] > b0 || (bv[q] == b0 && bi[q] < i0)) { b0 = bv[q]; i0 = bi[q]; }
            sp = i0 < n ? i0 : kk;
            piv[kk] = sp;
        }
        __syncthreads();
        const int p = sp;
        if (p != kk)
            for (int j = t; j < n; j += nt) {
                const double a = S[(int64_t)kk * n + j];
                S[(int64_t)kk * n + j] = S[(int64_t)p * n + j];
                S[(int64_t)p * n + j] = a;
            }
        __syncthreads();
        const double d = S[(int64_t)kk * n + kk];
        if (d == 0.0) {
            if (t == 0) bad[0] = 1;
            return;
        }
        for (int i = kk + 1 + t; i < n; i += nt) S[(int64_t)i * n + kk] /= d;
        __syncthreads();
        const int wr = k0 + w - kk - 1;  // panel columns right of kk
        if (wr > 0) {
            const int64_t tot = (int64_t)(n - kk - 1) * wr;
            for (int64_t e = t; e < tot; e += nt) {
                const int i = kk + 1 + (int)(e / wr), j = kk + 1 + (int)(e % wr);
                S[(int64_t)i * n + j] -= S[(int64_t)i * n + kk] * S[(int64_t)kk * n + j];
            }
        }
        __syncthreads();
    }
}

// X[r0 + r][c] for r < w, c in [c0, c1): solve with the w x w diagonal
// block T of row-major T (rows/cols starting at d0): UNIT lower forward
// substitution, else upper backward substitution with division by the
// diagonal.  One thread per column, the column held in registers.
template <bool LOWER>
__global__ __launch_bounds__(256) void k_trsm_block(int w, const double* __restrict__ T, int64_t ldt, int d0,
                                                    double* X, int64_t ldx, int r0, int c0, int c1) {
    __shared__ double Ts[kPanel][kPanel + 1];
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        const int a = e / w, b = e % w;
        Ts[a][b] = T[(int64_t)(d0 + a) * ldt + d0 + b];
    }
    __syncthreads();
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    double x[kPanel];
#pragma unroll
    for (int r = 0; r < kPanel; ++r) x[r] = r < w ? X[(int64_t)(r0 + r) * ldx + c] : 0.0;
    if (LOWER) {
#pragma unroll
        for (int r = 1; r < kPanel; ++r) {
            if (r < w) {
                double s = x[r];
#pragma unroll
                for (int q = 0; q < r; ++q) s -= Ts[r][q] * x[q];
                x[r] = s;
            }
        }
    } else {
#pragma unroll
        for (int r = kPanel - 1; r >= 0; --r) {
            if (r < w) {
                double s = x[r];
#pragma unroll
                for (int q = r + 1; q < kPanel; ++q)
                    if (q < w) s -= Ts[r][q] * x[q];
                x[r] = s / Ts[r][r];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kPanel; ++r)
        if (r < w) X[(int64_t)(r0 + r) * ldx + c] = x[r];
}
void launch_trsm_block(bool lower, int w, const double* T, int64_t ldt, int d0, double* X, int64_t ldx, int r0,
                       int c0, int c1, hipStream_t s) {
    if (c1 <= c0 || w <= 0) return;
    const int g = (c1 - c0 + 255) / 256;
    if (lower) k_trsm_block<true><<<g, 256, 0, s>>>(w, T, ldt, d0, X, ldx, r0, c0, c1);
    else k_trsm_block<false><<<g, 256, 0, s>>>(w, T, ldt, d0, X, ldx, r0, c0, c1);
}
void launch_lu_panel(int n, int k0, int w, double* S, int* piv, int* bad, hipStream_t s) {
    k_lu_panel<<<1, 1024, 0, s>>>(n, k0, w, S, piv, bad);
}

// Y = P (row i of Y is row o[i] of the identity)
__global__ void k_perm_identity(int n, const int* __restrict__ o, double* Y) {
    const int64_t tot = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        Y[e] = (j == o[i]) ? 1.0 : 0.0;
    }
}
void launch_perm_identity(int n, const int* o, double* Y, hipStream_t s) {
    k_perm_identity<<<4096, 256, 0, s>>>(n, o, Y);
}

// ------------------------------------------------------------------ tails
// Dense initialisation from the operator: Out[at[e]] = v[pos[e]] (the
// positions of E, F and C entries in the CSR, found once per pattern).
__global__ void k_scatter_from(int64_t m, const int64_t* __restrict__ pos, const int64_t* __restrict__ at,
                               const double* __restrict__ v, double* Out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        Out[at[e]] = v[pos[e]];
}
void launch_scatter_from(int64_t m, const int64_t* pos, const int64_t* at, const double* v, double* Out,
                         hipStream_t s) {
    if (m > 0) k_scatter_from<<<(int)std::min<int64_t>(4096, (m + 255) / 256), 256, 0, s>>>(m, pos, at, v, Out);
}

// H_b = L_TT^{-1} H_b in place, column by column (one thread per column):
// rows r = 0..t-1 of the tail (global row tail + r), the strict-lower
// entries of L at columns >= tail, ascending, subtracted one by one.
__global__ __launch_bounds__(256) void k_tail_lsolve(const TailDev T, const int* __restrict__ lrp,
                                                     const int* __restrict__ lci, const double* __restrict__ lval) {
    const int b = blockIdx.y;
    const int ne = T.ne[b];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ne) return;
    const int tail = T.tail[b], hi = T.bp[b + 1];
    double* H = T.H + T.hoff[b];
    for (int i = tail; i < hi; ++i) {
        double s = H[(int64_t)(i - tail) * ne + c];
        for (int q = lrp[i]; q < lrp[i + 1]; ++q) {
            const int j = lci[q];
            if (j >= tail) s -= lval[q] * H[(int64_t)(j - tail) * ne + c];
        }
        H[(int64_t)(i - tail) * ne + c] = s;
    }
}
// Gt_b = (F U_TT^{-1})^T in place, one thread per border row (column c of
// Gt): rows i ascending, g_i = f_i / u_ii, then f_j -= g_i u_ij for the
// strict-upper entries of row i.
__global__ __launch_bounds__(256) void k_tail_usolve(const TailDev T, const int* __restrict__ urp,
                                                     const int* __restrict__ uci, const double* __restrict__ uval,
                                                     const double* __restrict__ udiag) {
    const int b = blockIdx.y;
    const int nf = T.nf[b];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nf) return;
    const int tail = T.tail[b], hi = T.bp[b + 1];
    double* G = T.G + T.goff[b];
    for (int i = tail; i < hi; ++i) {
        const double g = G[(int64_t)(i - tail) * nf + c] / udiag[i];
        G[(int64_t)(i - tail) * nf + c] = g;
        if (g != 0.0)
            for (int q = urp[i]; q < urp[i + 1]; ++q) {
                const int j = uci[q];   // > i, inside the tail
                G[(int64_t)(j - tail) * nf + c] -= uval[q] * g;
            }
    }
}
void launch_tail_solves(const TailDev& T, int nblocks, int max_ne, int max_nf, const int* lrp, const int* lci,
                        const double* lval, const int* urp, const int* uci, const double* uval,
                        const double* udiag, hipStream_t s) {
    if (nblocks <= 0) return;
    if (max_ne > 0) k_tail_lsolve<<<dim3((max_ne + 255) / 256, nblocks), 256, 0, s>>>(T, lrp, lci, lval);
    if (max_nf > 0) k_tail_usolve<<<dim3((max_nf + 255) / 256, nblocks), 256, 0, s>>>(T, urp, uci, uval, udiag);
}

// ------------------------------------------------------------------ apply
// gpart[goff_v[b] + c] = sum_r Gt_b[r][c] w[tail_b + r]  (one thread per c)
__global__ __launch_bounds__(256) void k_tail_gt_w(const TailDev T, const double* __restrict__ w,
                                                   double* __restrict__ gpart) {
    const int b = blockIdx.y;
    const int nf = T.nf[b];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nf) return;
    const int tail = T.tail[b], hi = T.bp[b + 1];
    const double* G = T.G + T.goff[b];
    double s = 0.0;
    for (int r = 0; r < hi - tail; ++r) s = fma(G[(int64_t)r * nf + c], w[tail + r], s);
    gpart[T.fvoff[b] + c] = s;
}
// g[f] = r_border[f] - sum over the blocks touching border row f (block
// order) of their partial
__global__ void k_border_gather(int nbd, const int* __restrict__ fptr, const int* __restrict__ fidx,
                                const double* __restrict__ gpart, const double* __restrict__ rb,
                                double* __restrict__ g) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nbd; f += gridDim.x * blockDim.x) {
        double s = rb[f];
        for (int q = fptr[f]; q < fptr[f + 1]; ++q) s -= gpart[fidx[q]];
        g[f] = s;
    }
}
// x = A g for a dense row-major n x n A: one wave per row, DPP-free wave
// reduction in a fixed order
__global__ __launch_bounds__(256) void k_dense_gemv(int n, const double* __restrict__ A, const double* __restrict__ g,
                                                    double* __restrict__ x) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    for (int i = wave; i < n; i += nw) {
        double s = 0.0;
        for (int j = lane; j < n; j += kWave) s = fma(A[(int64_t)i * n + j], g[j], s);
        s = wave_sum(s);
        if (lane == 0) x[i] = s;
    }
}
// w[tail + r] -= sum_c H_b[r][c] x[ecols_b[c]]  (one wave per tail row)
__global__ __launch_bounds__(256) void k_tail_h_x(const TailDev T, int nblocks, const double* __restrict__ x,
                                                  double* __restrict__ w) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, lane = threadIdx.x % kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    for (int row = wave; row < T.ntail; row += nw) {
        // block of this tail row: tail rows are numbered block after block
        int lo = 0, hi = nblocks;
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (T.trow[mid] <= row) lo = mid;
            else hi = mid;
        }
        const int b = lo, r = row - T.trow[b];
        const int ne = T.ne[b];
        const double* H = T.H + T.hoff[b] + (int64_t)r * ne;
        const int* ec = T.ecols + T.ecoff[b];
        double s = 0.0;
        for (int c = lane; c < ne; c += kWave) s = fma(H[c], x[ec[c]], s);
        s = wave_sum(s);
        if (lane == 0) w[T.tail[b] + r] -= s;
    }
}
void launch_bbd_mid(const TailDev& T, int nblocks, int max_nf, int nbd, const double* Sinv, const int* fptr,
                    const int* fidx, double* gpart, const double* rb, double* g, double* w, double* xb,
                    hipStream_t s) {
    if (nblocks > 0 && max_nf > 0) k_tail_gt_w<<<dim3((max_nf + 255) / 256, nblocks), 256, 0, s>>>(T, w, gpart);
    k_border_gather<<<std::max(1, std::min(1024, (nbd + 255) / 256)), 256, 0, s>>>(nbd, fptr, fidx, gpart, rb, g);
    k_dense_gemv<<<std::max(1, std::min(4096, (nbd + 3) / 4)), 256, 0, s>>>(nbd, Sinv, g, xb);
    if (T.ntail > 0) k_tail_h_x<<<std::min(8192, (T.ntail + 3) / 4), 256, 0, s>>>(T, nblocks, xb, w);
}

}  // namespace sdsl
