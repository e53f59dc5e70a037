// Petrov-Galerkin projection of a reduced system onto the spaces the
// interpolation method builds (Section 1, the spaces V_k and W_k; Section 2:
// in controller-Hessenberg coordinates W^T A V - lambda W^T V equals
// What^T H Vhat - lambda What^T Vhat, and orthogonalising the columns of
// V_k, W_k is the same as orthogonalising those of Vhat, What).
//
//   1. real bases: column k of Vr is the real or the imaginary part of a
//      column of the complex V (the caller pairs conjugate points), likewise Wr;
//   2. orthonormal columns by classical Gram-Schmidt with one
//      reorthogonalisation (each pass projects against all earlier columns
//      at once), spread over workgroups that own ranges of rows;
//   3. Ar = Wr^T (H Vr), Er = Wr^T Vr, Br = Wr^T R, Cr = Ct Vr as FP64 GEMMs on
//      the matrix cores (R is nonzero in its first m rows only, so Br needs m
//      rows of Wr).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "shiftsolve.h"
#include "handle.hpp"

namespace shs {

namespace {

constexpr size_t kProjPart = (size_t)1 << 22;   // split-K partials (doubles)

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Vr(:, k) = Re or Im of V(:, sel[k] / 2) (even sel: real part), same for W
__global__ __launch_bounds__(256) void realify_kernel(int n, int r, const double *V, int64_t ldv, const double *W,
                                                      int64_t ldw, const int32_t *sel, double *Vr, double *Wr)
{
    const int k = blockIdx.y, which = blockIdx.z;
    const double *Z = which ? W : V;
    const int64_t ld = which ? ldw : ldv;
    double *out = (which ? Wr : Vr) + (int64_t)k * n;
    const int col = sel[k] >> 1, part = sel[k] & 1;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        out[i] = Z[((int64_t)col * ld + i) * 2 + part];
}

// Classical Gram-Schmidt with one reorthogonalisation, spread over the
// chip: for column k of either basis, two passes of
// v <- v - Q(:, 0:k) (Q(:, 0:k)^T v), then v <- v / ||v||.  Both bases go
// through the same launches (blockIdx.y); each workgroup owns a fixed range
// of rows, and a pass is two launches: partial dot products of its rows
// against the earlier columns (cgs_dot_kernel), then every workgroup sums
// the partials in the same fixed order and updates its rows
// (cgs_update_kernel).  The second update also leaves partial squared
// norms, from which the next column's first launch (or cgs_scale_kernel
// after the last column) scales column k.  A column that vanishes in exact
// arithmetic (norm below 2^-40 of its norm before the passes) becomes zeros
// and is flagged in *flag.  Four launches per column, no host waits.
constexpr int kCgsThreads = 256;
constexpr int kCgsRowsMin = 512;   // rows per workgroup, at least
constexpr int kCgsChunk = 16;      // dot products reduced together
constexpr int kCgsCoef = 256;      // coefficients staged in LDS at a time

struct CgsArgs {
    int n, r, rows, G;       // rows per workgroup, workgroups per basis
    double *Q0, *Q1;         // n x r, ld n
    double *part;            // [2][G][r] partial dot products of the current pass
    double *nrm;             // [2][2][G][2] by column parity, basis, workgroup: partial
                             // ||v||^2 before the passes, after them
    int *flag;
};

// Sum of one value over the workgroup, the same order in every workgroup.
__device__ inline double cgs_block_sum(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kCgsThreads / 64; ++q) s += red[q];
    return s;
}

// sum over the G workgroups' partials x[g * stride], fixed order
__device__ inline double cgs_partials(const double *x, int G, int stride, double *red)
{
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += kCgsThreads) s += x[(int64_t)g * stride];
    return cgs_block_sum(s, red);
}

// The partial norms of column k and basis b.  Column k's first launch
// writes them while other workgroups of the same launch still read column
// k-1's, hence two sets by column parity.
__device__ inline double *cgs_nrm(const CgsArgs &a, int k, int b)
{
    return a.nrm + ((int64_t)(k & 1) * 2 + b) * a.G * 2;
}

// Scale column k of basis b on this workgroup's rows (every workgroup
// computes the same norms from the same partials).
__device__ inline void cgs_scale(const CgsArgs &a, int b, int k, double *red)
{
    double *Q = b ? a.Q1 : a.Q0;
    const double *nb = cgs_nrm(a, k, b);
    const double nrm0 = sqrt(cgs_partials(nb, a.G, 2, red));
    const double nrm = sqrt(cgs_partials(nb + 1, a.G, 2, red));
    const bool dead = !(nrm > 0x1p-40 * nrm0);
    const double sc = dead ? 0.0 : 1.0 / nrm;
    double *v = Q + (int64_t)k * a.n;
    const int i0 = blockIdx.x * a.rows, i1 = min(a.n, i0 + a.rows);
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kCgsThreads) v[i] = dead ? 0.0 : v[i] * sc;
    if (dead && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(a.flag, 1);
}

// Partial dot products of column k against columns 0 .. k-1 over this
// workgroup's rows; in the first pass also its partial ||v||^2, after
// scaling column k-1 (the rows this thread reads below are the ones it
// scales).
__global__ __launch_bounds__(kCgsThreads) void cgs_dot_kernel(CgsArgs a, int k, int first)
{
    __shared__ double red[kCgsThreads / 64];
    __shared__ double sums[kCgsChunk];
    const int b = blockIdx.y, g = blockIdx.x, t = threadIdx.x;
    if (first && k > 0) cgs_scale(a, b, k - 1, red);
    const double *Q = b ? a.Q1 : a.Q0;
    const double *v = Q + (int64_t)k * a.n;
    const int i0 = g * a.rows, i1 = min(a.n, i0 + a.rows);
    double *pp = a.part + ((int64_t)b * a.G + g) * a.r;
    for (int j0 = 0; j0 < k; j0 += kCgsChunk) {
        const int nj = min(kCgsChunk, k - j0);
        double acc[kCgsChunk];
#pragma unroll
        for (int q = 0; q < kCgsChunk; ++q) acc[q] = 0.0;
        for (int i = i0 + t; i < i1; i += kCgsThreads) {
            const double vi = v[i];
#pragma unroll
            for (int q = 0; q < kCgsChunk; ++q)
                if (q < nj) acc[q] = fma(Q[(int64_t)(j0 + q) * a.n + i], vi, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < kCgsChunk; ++q) {
            const double s = cgs_block_sum(acc[q], red);
            if (t == 0) sums[q] = s;
        }
        __syncthreads();
        if (t < nj) pp[j0 + t] = sums[t];
        __syncthreads();
    }
    if (first) {
        double s = 0.0;
        for (int i = i0 + t; i < i1; i += kCgsThreads) s = fma(v[i], v[i], s);
        s = cgs_block_sum(s, red);
        if (t == 0) cgs_nrm(a, k, b)[g * 2] = s;
    }
}

// v <- v - Q(:, 0:k) c over this workgroup's rows, c the summed partials;
// after the second pass also its partial ||v||^2.
__global__ __launch_bounds__(kCgsThreads) void cgs_update_kernel(CgsArgs a, int k, int last)
{
    __shared__ double red[kCgsThreads / 64];
    __shared__ double c[kCgsCoef];
    const int b = blockIdx.y, g = blockIdx.x, t = threadIdx.x;
    double *Q = b ? a.Q1 : a.Q0;
    double *v = Q + (int64_t)k * a.n;
    const int i0 = g * a.rows, i1 = min(a.n, i0 + a.rows);
    const double *pb = a.part + (int64_t)b * a.G * a.r;
    for (int j0 = 0; j0 < k; j0 += kCgsCoef) {
        const int nj = min(kCgsCoef, k - j0);
        __syncthreads();   // the previous chunk's coefficients are no longer read
        if (t < nj) {
            double s = 0.0;
            for (int q = 0; q < a.G; ++q) s += pb[(int64_t)q * a.r + j0 + t];
            c[t] = s;
        }
        __syncthreads();
        for (int i = i0 + t; i < i1; i += kCgsThreads) {
            double vi = v[i];
            for (int q = 0; q < nj; ++q) vi = fma(-c[q], Q[(int64_t)(j0 + q) * a.n + i], vi);
            v[i] = vi;
        }
    }
    if (last) {
        double s = 0.0;
        for (int i = i0 + t; i < i1; i += kCgsThreads) s = fma(v[i], v[i], s);
        s = cgs_block_sum(s, red);
        if (t == 0) cgs_nrm(a, k, b)[g * 2 + 1] = s;
    }
}

__global__ __launch_bounds__(kCgsThreads) void cgs_scale_kernel(CgsArgs a, int k)
{
    __shared__ double red[kCgsThreads / 64];
    cgs_scale(a, blockIdx.y, k, red);
}

// Workgroups per basis: rows of at least kCgsRowsMin per workgroup, and the
// partials within the buffer of `cap` doubles.
inline int cgs_groups(int64_t n, int64_t r, size_t cap)
{
    const int64_t by_rows = (n + kCgsRowsMin - 1) / kCgsRowsMin;
    const int64_t by_buf = (int64_t)(cap / (size_t)(2 * r + 8));
    return (int)std::max<int64_t>(1, std::min(by_rows, by_buf));
}

hipError_t cgs2(int n, int r, double *Q0, double *Q1, double *part, size_t cap, int *flag, hipStream_t st)
{
    CgsArgs a{};
    a.n = n;
    a.r = r;
    a.G = cgs_groups(n, r, cap);
    a.rows = (n + a.G - 1) / a.G;
    a.Q0 = Q0;
    a.Q1 = Q1;
    a.part = part;
    a.nrm = part + (size_t)2 * a.G * r;
    a.flag = flag;
    const dim3 grid((unsigned)a.G, 2);
    for (int k = 0; k < r; ++k) {
        hipLaunchKernelGGL(cgs_dot_kernel, grid, dim3(kCgsThreads), 0, st, a, k, 1);
        hipLaunchKernelGGL(cgs_update_kernel, grid, dim3(kCgsThreads), 0, st, a, k, 0);
        hipLaunchKernelGGL(cgs_dot_kernel, grid, dim3(kCgsThreads), 0, st, a, k, 0);
        hipLaunchKernelGGL(cgs_update_kernel, grid, dim3(kCgsThreads), 0, st, a, k, 1);
    }
    hipLaunchKernelGGL(cgs_scale_kernel, grid, dim3(kCgsThreads), 0, st, a, r - 1);
    return hipGetLastError();
}

struct ProjLayout {
    size_t vr = 0, wr = 0, hv = 0, part = 0, flag = 0, total = 0;
};

ProjLayout proj_layout(int64_t n, int64_t r)
{
    ProjLayout L;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += al256(b); return o; };
    L.vr = take(sizeof(double) * n * r);
    L.wr = take(sizeof(double) * n * r);
    L.hv = take(sizeof(double) * n * r);
    L.part = take(sizeof(double) * kProjPart);
    L.flag = take(8);   // cleared as 8 bytes
    L.total = off;
    return L;
}

template <typename T>
inline T *atb(void *base, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }

}  // namespace

}  // namespace shs

using namespace shs;

extern "C" int shs_project_workspace(const shs_handle *h, int64_t r, size_t *bytes)
{
    if (!h) return -1;
    if (r < 1 || r > h->n) return -2;
    if (!bytes) return -3;
    *bytes = proj_layout(h->n, r).total;
    return 0;
}

extern "C" int shs_project(shs_handle *h, int64_t r, const double *V, int64_t ldv, const double *W, int64_t ldw,
                           const int32_t *sel, void *work, size_t work_bytes, double *Ar, double *Er, double *Br,
                           double *Cr, int32_t *rank_def, void *stream)
{
    if (!h) return -1;
    if (r < 1 || r > h->n || r > 65535) return -2;
    if (!V) return -3;
    if (ldv < h->n) return -4;
    if (!W) return -5;
    if (ldw < h->n) return -6;
    if (!sel) return -7;
    if (!Ar) return -10;
    if (!Er) return -11;
    if (!Br) return -12;
    if (h->p > 0 && !Cr) return -13;
    if (!rank_def) return -14;
    const int64_t n = h->n, m = h->m, p = h->p;
    const ProjLayout L = proj_layout(n, r);
    hipStream_t st = (hipStream_t)stream;
    bool owned = false;
    if (work) {
        if (work_bytes < L.total) return -9;
    } else {
        if (hipMallocAsync(&work, L.total, st) != hipSuccess) return SHS_ERR_NOMEM;
        owned = true;
    }
    double *Vr = atb<double>(work, L.vr), *Wr = atb<double>(work, L.wr), *HV = atb<double>(work, L.hv);
    double *part = atb<double>(work, L.part);
    int *flag = atb<int>(work, L.flag);
    hipError_t e = zero_fill(flag, 8, st);
    hipLaunchKernelGGL(realify_kernel, dim3(std::max<unsigned>(1, std::min<unsigned>(64, (unsigned)((n + 255) / 256))),
                                            (unsigned)r, 2),
                       dim3(256), 0, st, (int)n, (int)r, V, ldv, W, ldw, sel, Vr, Wr);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = cgs2((int)n, (int)r, Vr, Wr, part, kProjPart, flag, st);
    // Ar = Wr^T (H Vr), Er = Wr^T Vr, Br = Wr(0:m, :)^T R(0:m, :), Cr = Ct Vr
    if (e == hipSuccess)
        e = dgemm(false, false, (int)n, (int)r, (int)n, 1.0, h->H, h->ldh, Vr, n, HV, n, false, part, kProjPart, st);
    if (e == hipSuccess)
        e = dgemm(true, false, (int)r, (int)r, (int)n, 1.0, Wr, n, HV, n, Ar, r, false, part, kProjPart, st);
    if (e == hipSuccess)
        e = dgemm(true, false, (int)r, (int)r, (int)n, 1.0, Wr, n, Vr, n, Er, r, false, part, kProjPart, st);
    if (e == hipSuccess)
        e = dgemm(true, false, (int)r, (int)m, (int)m, 1.0, Wr, n, h->Bw, n, Br, r, false, nullptr, 0, st);
    if (e == hipSuccess && p > 0)
        e = dgemm(false, false, (int)p, (int)r, (int)n, 1.0, h->Ct, h->ldct, Vr, n, Cr, p, false, part, kProjPart,
                     st);
    if (e == hipSuccess) e = hipMemcpyAsync(rank_def, flag, sizeof(int), hipMemcpyDeviceToDevice, st);
    if (owned) {
        const hipError_t e2 = hipFreeAsync(work, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SHS_ERR_NOMEM : SHS_ERR_HIP;
    return 0;
}
