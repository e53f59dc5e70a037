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
//      at once), one workgroup per basis;
//   3. Ar = Wr^T (H Vr), Er = Wr^T Vr, Br = Wr^T R, Cr = Ct Vr as FP64 GEMMs on
//      the matrix cores (R is nonzero in its first m rows only, so Br needs m
//      rows of Wr).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "shiftsolve.h"
#include "handle.hpp"

namespace shs {

namespace {

constexpr int kOrthoThreads = 1024;
constexpr int kOrthoChunk = 16;   // coefficients reduced together
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

__device__ inline double block_sum(double v, double *red)
{
    // wave sums, then the first wave sums the 16 wave results
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = l < kOrthoThreads / 64 ? red[l] : 0.0;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    return t;   // every thread holds the total
}

// Orthonormalise the r columns of Q (n x r, ld n) in place: for each column,
// two passes of v <- v - Q(:, 0:k) (Q(:, 0:k)^T v), then v <- v / ||v||.  A
// column that vanishes in exact arithmetic (norm below 2^-40 of its norm
// before the passes) is returned as zeros and flagged in *rank_def.
__global__ __launch_bounds__(kOrthoThreads) void cgs2_kernel(int n, int r, double *Q0, double *Q1, int *rank_def)
{
    double *Q = blockIdx.x == 0 ? Q0 : Q1;
    __shared__ double red[kOrthoThreads / 64];
    __shared__ double part[kOrthoThreads / 64][kOrthoChunk];
    __shared__ double coef[kOrthoChunk];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int k = 0; k < r; ++k) {
        double *v = Q + (int64_t)k * n;
        double nrm0 = 0.0;
        for (int i = t; i < n; i += kOrthoThreads) nrm0 = fma(v[i], v[i], nrm0);
        nrm0 = sqrt(block_sum(nrm0, red));
        for (int pass = 0; pass < 2; ++pass) {
            for (int j0 = 0; j0 < k; j0 += kOrthoChunk) {
                const int nj = min(kOrthoChunk, k - j0);
                double acc[kOrthoChunk];
#pragma unroll
                for (int q = 0; q < kOrthoChunk; ++q) acc[q] = 0.0;
                for (int i = t; i < n; i += kOrthoThreads) {
                    const double vi = v[i];
#pragma unroll
                    for (int q = 0; q < kOrthoChunk; ++q)
                        if (q < nj) acc[q] = fma(Q[(int64_t)(j0 + q) * n + i], vi, acc[q]);
                }
#pragma unroll
                for (int q = 0; q < kOrthoChunk; ++q) {
                    double a = acc[q];
                    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
                    if (l == 0) part[w][q] = a;
                }
                __syncthreads();
                if (t < nj) {
                    double s = 0.0;
                    for (int q = 0; q < kOrthoThreads / 64; ++q) s += part[q][t];
                    coef[t] = s;
                }
                __syncthreads();
                // classical Gram-Schmidt within the chunk: the coefficients of
                // the chunk were all taken from the same v
                for (int i = t; i < n; i += kOrthoThreads) {
                    double vi = v[i];
                    for (int q = 0; q < nj; ++q) vi = fma(-coef[q], Q[(int64_t)(j0 + q) * n + i], vi);
                    v[i] = vi;
                }
                __syncthreads();
            }
        }
        double nrm = 0.0;
        for (int i = t; i < n; i += kOrthoThreads) nrm = fma(v[i], v[i], nrm);
        nrm = sqrt(block_sum(nrm, red));
        const bool dead = !(nrm > 0x1p-40 * nrm0);
        const double sc = dead ? 0.0 : 1.0 / nrm;
        for (int i = t; i < n; i += kOrthoThreads) v[i] = dead ? 0.0 : v[i] * sc;
        if (dead && t == 0) atomicOr(rank_def, 1);
        __syncthreads();
    }
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
    hipLaunchKernelGGL(cgs2_kernel, dim3(2), dim3(kOrthoThreads), 0, st, (int)n, (int)r, Vr, Wr, flag);
    if (e == hipSuccess) e = hipGetLastError();
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
