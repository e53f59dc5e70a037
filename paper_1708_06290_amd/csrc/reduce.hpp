// Controller-Hessenberg reduction (Algorithm 1, Section 2) on the GPU, FP64.
//
//   1. QR of B by Householder reflectors P_j (j < m, acting on rows j..n-1);
//   2. A <- P_j A P_j and C <- C P_j for each of them (the similarity with
//      Q_B);
//   3. for j = 0 .. n-m-2 a reflector on rows j+m .. n-1 annihilates
//      A(j+m+1 : n, j), applied from both sides and to C (Section 2.1 uses
//      the same reflectors, accumulated in blocks);
//   4. a diagonal sign matrix S makes R(i,i) >= 0 and H(j+m, j) >= 0.
//
// The kernels here are the unblocked building blocks: one reflector per
// column (a single workgroup reduces the column), a left update with one
// workgroup per column (a column is contiguous in column-major storage, so
// the dot product and the rank-1 update read it coalesced), and a right
// update split into partial dot products over column chunks followed by the
// rank-1 update.
#pragma once

#include "common.hpp"

namespace shs {

// Block-wide sum of a double over blockDim.x (<= 1024) threads.
__device__ inline double block_sum(double v, double *scratch)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

// Householder reflector of x (length L, contiguous): (I - tau v v^T) x = beta e_0,
// v_0 = 1, beta = -sign(x_0) ||x||.  Writes v (length L) to vout, tau to *tau,
// and overwrites x with (beta, 0, ..., 0).
__global__ __launch_bounds__(1024) void house_kernel(int L, double *x, double *vout, double *tau)
{
    __shared__ double scratch[16];
    // read before the barriers of block_sum: thread 0 overwrites x[0] below
    const double alpha = x[0];
    double part = 0.0;
    for (int i = 1 + threadIdx.x; i < L; i += blockDim.x) part = fma(x[i], x[i], part);
    const double sig2 = block_sum(part, scratch);
    if (sig2 == 0.0) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) vout[i] = (i == 0) ? 1.0 : 0.0;
        if (threadIdx.x == 0) *tau = 0.0;
        return;
    }
    const double nu = sqrt(fma(alpha, alpha, sig2));
    const double beta = alpha >= 0.0 ? -nu : nu;
    const double scal = 1.0 / (alpha - beta);
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        vout[i] = (i == 0) ? 1.0 : x[i] * scal;
        x[i] = (i == 0) ? beta : 0.0;
    }
    if (threadIdx.x == 0) *tau = (beta - alpha) / beta;
}

// Left update of columns c0 + blockIdx.x: A(r0:r0+L, c) -= tau v (v^T A(r0:r0+L, c)).
__global__ __launch_bounds__(256) void left_update_kernel(int L, int r0, int c0, double *A, int64_t lda,
                                                          const double *v, const double *tau)
{
    __shared__ double scratch[8];
    const double t = *tau;
    if (t == 0.0) return;
    double *col = A + (int64_t)(c0 + blockIdx.x) * lda + r0;
    double part = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) part = fma(v[i], col[i], part);
    const double w = block_sum(part, scratch) * t;
    for (int i = threadIdx.x; i < L; i += blockDim.x) col[i] = fma(-w, v[i], col[i]);
}

// Right update A(0:rows, c0:c0+L) -= tau (A v) v^T, phase 1: partial sums
// part[chunk * rows + i] = sum over the chunk's columns of A(i, c0+k) v_k.
constexpr int kRightChunk = 128;

__global__ __launch_bounds__(256) void right_dot_kernel(int rows, int L, int c0, const double *A, int64_t lda,
                                                        const double *v, const double *tau, double *part)
{
    if (*tau == 0.0) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int k0 = blockIdx.y * kRightChunk;
    const int k1 = min(L, k0 + kRightChunk);
    if (i >= rows) return;
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s = fma(A[(int64_t)(c0 + k) * lda + i], v[k], s);
    part[(int64_t)blockIdx.y * rows + i] = s;
}

// phase 2: u_i = sum of the partials; A(i, c0+k) -= tau u_i v_k for the chunk.
__global__ __launch_bounds__(256) void right_update_kernel(int rows, int L, int c0, double *A, int64_t lda,
                                                           const double *v, const double *tau,
                                                           const double *part, int nchunks)
{
    const double t = *tau;
    if (t == 0.0) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    double u = 0.0;
    for (int q = 0; q < nchunks; ++q) u += part[(int64_t)q * rows + i];
    u *= t;
    const int k0 = blockIdx.y * kRightChunk;
    const int k1 = min(L, k0 + kRightChunk);
    for (int k = k0; k < k1; ++k) {
        double *p = A + (int64_t)(c0 + k) * lda + i;
        *p = fma(-u, v[k], *p);
    }
}

// Sign normalisation: s_i = sign(R(i,i)) for i < m, s_{j+m} = sign(H(j+m,j) s_j).
// Serial over the chain (O(n)), one thread.
__global__ void signs_kernel(int n, int m, const double *H, int64_t ldh, const double *Bw, int64_t ldb,
                             double *sgn)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < m; ++i) sgn[i] = Bw[(int64_t)i * ldb + i] < 0.0 ? -1.0 : 1.0;
    for (int j = 0; j + m < n; ++j) {
        const double h = H[(int64_t)j * ldh + j + m] * sgn[j];
        sgn[j + m] = h < 0.0 ? -1.0 : 1.0;
    }
}

// H <- S H S (and exact zeros below the band), H32 = (float)H, row sums of
// |H(i, k)| for k != i, and the diagonal.  One thread per row.
__global__ __launch_bounds__(256) void finalize_h_kernel(int n, int m, double *H, int64_t ldh, float *H32,
                                                         const double *sgn, double *offrow, double *diag)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double si = sgn[i];
    double sum = 0.0;
    for (int k = 0; k < n; ++k) {
        double *p = H + (int64_t)k * ldh + i;
        double h = (i > k + m) ? 0.0 : (*p) * si * sgn[k];
        *p = h;
        H32[(int64_t)k * ldh + i] = (float)h;
        if (k != i) sum += fabs(h);
        else diag[i] = h;
    }
    offrow[i] = sum;
}

// R <- S R (rows >= m zero, strictly lower part zero), Rtop = R(0:m, 0:m),
// column maxima of |R|; Ct <- Ct S.
__global__ void finalize_r_kernel(int n, int m, double *Bw, int64_t ldb, const double *sgn,
                                  double *Rtop, double *rcolmax)
{
    const int c = threadIdx.x;
    if (c >= m) return;
    double mx = 0.0;
    for (int i = 0; i < n; ++i) {
        double *p = Bw + (int64_t)c * ldb + i;
        const double v = (i < m && i <= c) ? (*p) * sgn[i] : 0.0;
        *p = v;
        if (i < m) Rtop[c * m + i] = v;
        mx = fabs(v) > mx ? fabs(v) : mx;
    }
    rcolmax[c] = mx;
}

__global__ __launch_bounds__(256) void scale_cols_kernel(int rows, int n, double *Ct, int64_t ldc,
                                                         const double *sgn)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)rows * n) return;
    const int64_t k = idx / rows, r = idx % rows;
    Ct[k * ldc + r] *= sgn[k];
}

// X (complex, n x ncols, ld) <- diag(s) X
__global__ __launch_bounds__(256) void scale_rows_complex_kernel(int n, int ncols, double *X, int64_t ld,
                                                                 const double *sgn)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * ncols) return;
    const int64_t c = idx / n, i = idx % n;
    double *p = X + (c * ld + i) * 2;
    p[0] *= sgn[i];
    p[1] *= sgn[i];
}

// X(r0:r0+L, :) -= tau v (v^T X(r0:r0+L, :)) for complex X; one workgroup per column.
__global__ __launch_bounds__(256) void reflect_complex_kernel(int L, int r0, double *X, int64_t ld,
                                                              const double *v, const double *tau)
{
    __shared__ double scratch[8];
    const double t = *tau;
    if (t == 0.0) return;
    double *col = X + ((int64_t)blockIdx.x * ld + r0) * 2;
    double pr = 0.0, pi = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        pr = fma(v[i], col[2 * i], pr);
        pi = fma(v[i], col[2 * i + 1], pi);
    }
    const double wr = block_sum(pr, scratch) * t;
    const double wi = block_sum(pi, scratch) * t;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        col[2 * i] = fma(-wr, v[i], col[2 * i]);
        col[2 * i + 1] = fma(-wi, v[i], col[2 * i + 1]);
    }
}

__global__ __launch_bounds__(256) void copy_complex_kernel(int n, int ncols, const double *src, int64_t lds,
                                                           double *dst, int64_t ldd)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * ncols) return;
    const int64_t c = idx / n, i = idx % n;
    dst[(c * ldd + i) * 2] = src[(c * lds + i) * 2];
    dst[(c * ldd + i) * 2 + 1] = src[(c * lds + i) * 2 + 1];
}

// ---------------------------------------------------------------------------
// Blocked m-Hessenberg reduction (Algorithms 2 and 3): one panel of b
// columns at a time, split into mini-blocks of m columns.  Before a
// mini-block runs, every earlier reflector of the panel has been applied to
// its columns by GEMMs (from the right: Y V^T with Y = A V T; from the left:
// (I - V T^T V^T)); this kernel finishes the columns with the mini-block's
// own reflectors, one column after the other, on a single workgroup.
//
// A reflector of the mini-block acts on rows >= its column + m, and the
// mini-block has at most m columns, so its reflectors never touch its own
// columns from the right: only the left products are needed here.  Column
// jj gets them in compact form, x <- x - V_b T_b^T (V_b^T x) with V_b, T_b
// the mini-block's first jj reflectors and their triangular factor, in
// three passes over the column:
//   1. d = V_b^T x;
//   2. x <- x - V_b (T_b^T d), while summing ||x(r0+1:)||^2 and
//      e = V_b(r0+1:, :)^T x(r0+1:) (r0 = column + m, the reflector's first row);
//   3. the reflector v = (1, x(r0+1:) / (alpha - beta)) is written, x becomes
//      (beta, 0, ...).  Its T column follows from e without another pass:
//      V_b^T v = V_b(r0, :)^T + e / (alpha - beta).
//
//   columns j0 .. j0+mb-1 of A; rows r_lo .. n-1 are the ones the panel's
//   reflectors touch (r_lo = z + m for the panel starting at column z);
//   V: the panel's Householder vectors (column-major, ld n, absolute rows,
//   zeros above each vector's first row; rows < r_lo are not written);
//   taus: the panel's taus; T: the panel's b x b triangular factor (ld ldt),
//   of which this kernel writes the diagonal block of the mini-block
//   (columns q0 .. q0+mb-1).  Launch with 1024 threads.
constexpr int kMbNv = SHS_MAX_M + 1;

// Sums v[k] over the workgroup for k < cnt (cnt uniform); the totals land in
// tot[k].  Fixed order, so the result is reproducible.
__device__ inline void block_sum_multi(const double (&v)[kMbNv], int cnt, double (*red)[kMbNv], double *tot)
{
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < kMbNv; ++k) {
        if (k < cnt) {
            double s = v[k];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if ((threadIdx.x & 63) == 0) red[w][k] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[i][threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void miniblock_kernel(int n, int m, int r_lo, int j0, int mb, int q0, double *A,
                                                         int64_t lda, double *V, double *taus, double *T, int ldt)
{
    __shared__ double red[16][kMbNv];
    __shared__ double tot[kMbNv];
    __shared__ double Ts[SHS_MAX_M][SHS_MAX_M];   // Ts[l][k] = T(q0 + l, q0 + k)
    __shared__ double wv[SHS_MAX_M];
    __shared__ double s_alpha;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double *Vb = V + (int64_t)q0 * n;
    for (int e = tid; e < SHS_MAX_M * SHS_MAX_M; e += nt) Ts[e / SHS_MAX_M][e % SHS_MAX_M] = 0.0;
    __syncthreads();
    for (int jj = 0; jj < mb; ++jj) {
        const int j = j0 + jj, r0 = j + m;
        double *x = A + (int64_t)j * lda;
        // 1. d = V_b^T x, then w = T_b^T d
        if (jj > 0) {
            double d[kMbNv] = {};
            for (int i = r_lo + tid; i < n; i += nt) {
                const double xi = x[i];
#pragma unroll
                for (int l = 0; l < SHS_MAX_M; ++l)
                    if (l < jj) d[l] = fma(Vb[(int64_t)l * n + i], xi, d[l]);
            }
            block_sum_multi(d, jj, red, tot);
            if (tid < jj) {
                double s = 0.0;
                for (int k = 0; k <= tid; ++k) s = fma(Ts[k][tid], tot[k], s);
                wv[tid] = s;
            }
            __syncthreads();
        }
        // 2. x <- x - V_b w; sig2 = ||x(r0+1:)||^2 and e = V_b(r0+1:, :)^T x(r0+1:)
        double acc[kMbNv] = {};
        for (int i = r_lo + tid; i < n; i += nt) {
            double xi = x[i];
            if (jj > 0) {
#pragma unroll
                for (int l = 0; l < SHS_MAX_M; ++l)
                    if (l < jj) xi = fma(-wv[l], Vb[(int64_t)l * n + i], xi);
                x[i] = xi;
            }
            if (i == r0) s_alpha = xi;
            if (i > r0) {
                acc[0] = fma(xi, xi, acc[0]);
#pragma unroll
                for (int l = 0; l < SHS_MAX_M; ++l)
                    if (l < jj) acc[1 + l] = fma(Vb[(int64_t)l * n + i], xi, acc[1 + l]);
            }
        }
        block_sum_multi(acc, jj + 1, red, tot);
        const double sig2 = tot[0];
        const double alpha = s_alpha;
        double *vout = V + (int64_t)(q0 + jj) * n;
        double tau = 0.0, scal = 0.0;
        // 3. the reflector and the new column
        if (sig2 == 0.0) {
            for (int i = r_lo + tid; i < n; i += nt) vout[i] = (i == r0) ? 1.0 : 0.0;
        } else {
            const double nu = sqrt(fma(alpha, alpha, sig2));
            const double beta = alpha >= 0.0 ? -nu : nu;
            scal = 1.0 / (alpha - beta);
            tau = (beta - alpha) / beta;
            for (int i = r_lo + tid; i < n; i += nt) {
                if (i < r0) {
                    vout[i] = 0.0;
                } else if (i == r0) {
                    vout[i] = 1.0;
                    x[i] = beta;
                } else {
                    vout[i] = x[i] * scal;
                    x[i] = 0.0;
                }
            }
        }
        // T column: T(l, jj) = -tau sum_{l <= k < jj} T(l, k) (v_k . v),  T(jj, jj) = tau
        if (tid < jj) wv[tid] = Vb[(int64_t)tid * n + r0] + scal * tot[1 + tid];   // v_tid . v
        __syncthreads();
        if (tid < jj) {
            double s = 0.0;
            for (int k = tid; k < jj; ++k) s = fma(Ts[tid][k], wv[k], s);
            Ts[tid][jj] = -tau * s;
        }
        if (tid == 0) {
            taus[q0 + jj] = tau;
            Ts[jj][jj] = tau;
        }
        __syncthreads();
    }
    for (int e = tid; e < mb * mb; e += nt) {
        const int l = e % mb, k = e / mb;
        T[(int64_t)(q0 + k) * ldt + q0 + l] = Ts[l][k];
    }
}

}  // namespace shs
