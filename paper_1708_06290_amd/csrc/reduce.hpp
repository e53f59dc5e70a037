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
    double part = 0.0;
    for (int i = 1 + threadIdx.x; i < L; i += blockDim.x) part = fma(x[i], x[i], part);
    const double sig2 = block_sum(part, scratch);
    const double alpha = x[0];
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

}  // namespace shs
