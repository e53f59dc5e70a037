// Structured pseudospectrum: the spectral norm of the transfer function at
// every point of a set.
//
// Section 1: the structured epsilon-pseudospectrum of (A, B, C) is the set of
// points z with ||C (zI - A)^{-1} B||_2 >= 1/epsilon, i.e. the z that are
// eigenvalues of A + B E C for some perturbation with ||E||_2 <= epsilon.
// shs_solve's G_j = C (A - z_j I)^{-1} B differs from that function only in
// sign, so ||G_j||_2 is the quantity to threshold.
//
// ||G_j||_2 is the square root of the largest eigenvalue of the Hermitian
// Gram matrix G_j^* G_j (m x m) or G_j G_j^* (p x p), whichever is smaller
// (at most 16 x 16).  One wavefront per point: G_j is scaled by a power of
// two so that its largest entry lies in [1, 2) (no overflow or underflow in
// the Gram matrix, no rounding), the Gram matrix goes to LDS, and cyclic
// two-sided Jacobi sweeps with the round-robin pair order diagonalise it;
// the k/2 disjoint rotations of one round are applied together, first to the
// columns, then to the rows.  The largest eigenvalue is then accurate to a few
// units of rounding relative to ||G_j||_2^2.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "shiftsolve.h"
#include "common.hpp"

namespace shs {

namespace {

constexpr int kMaxK = SHS_MAX_M;
constexpr int kMaxSweeps = 40;

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Position of slot i in round r of the round-robin tournament on kk players
// (kk even): player 0 stays, the others rotate.
__device__ inline int rr_player(int i, int r, int kk) { return i == 0 ? 0 : 1 + (i - 1 + r) % (kk - 1); }

__global__ __launch_bounds__(64) void gnorm2_kernel(int p, int m, const double *G, int64_t ldg, double *out)
{
    __shared__ double a[2 * kMaxK * kMaxK];   // Gram matrix, (r, c) at 2 (c k + r)
    __shared__ double rot[kMaxK / 2][4];      // per pair: c, s, cos(phi), sin(phi)
    __shared__ int pa[kMaxK / 2], pb[kMaxK / 2], act[kMaxK / 2];
    const int j = blockIdx.x, t = threadIdx.x;
    const int k = min(p, m);
    const double *Gj = G + (int64_t)j * m * ldg * 2;   // G_j(i, c) at Gj[2 (c ldg + i)]
    // largest entry (NaN and infinity propagate as NaN)
    double mx = 0.0;
    bool bad = false;
    for (int e = t; e < p * m; e += kWave) {
        const int c = e / p, i = e - c * p;
        const double re = Gj[2 * ((int64_t)c * ldg + i)], im = Gj[2 * ((int64_t)c * ldg + i) + 1];
        const double v = fmax(fabs(re), fabs(im));
        if (!(fabs(re) <= DBL_MAX) || !(fabs(im) <= DBL_MAX)) bad = true;
        mx = fmax(mx, v);
    }
    mx = wave_max(mx);
    bad = __any(bad);
    if (bad) {
        if (t == 0) out[j] = __builtin_nan("");
        return;
    }
    if (mx == 0.0) {
        if (t == 0) out[j] = 0.0;
        return;
    }
    // exact scaling by a power of two: largest entry in [1, 2) (ldexp per
    // entry: 2^-ex itself overflows when G_j holds only subnormal numbers)
    const int ex = ilogb(mx);
    auto gs = [&](int i, int c, int part) { return ldexp(Gj[2 * ((int64_t)c * ldg + i) + part], -ex); };
    // Gram matrix of the scaled block
    const bool right = m <= p;   // G^* G (m x m), else G G^* (p x p)
    double fro = 0.0;
    for (int e = t; e < k * k; e += kWave) {
        const int c = e / k, r = e - c * k;
        double sr = 0.0, si = 0.0;
        if (right) {   // sum_i conj(G(i, r)) G(i, c)
            for (int i = 0; i < p; ++i) {
                const double xr = gs(i, r, 0), xi = gs(i, r, 1);
                const double yr = gs(i, c, 0), yi = gs(i, c, 1);
                sr = fma(xr, yr, fma(xi, yi, sr));
                si = fma(xr, yi, fma(-xi, yr, si));
            }
        } else {       // sum_q G(r, q) conj(G(c, q))
            for (int q = 0; q < m; ++q) {
                const double xr = gs(r, q, 0), xi = gs(r, q, 1);
                const double yr = gs(c, q, 0), yi = gs(c, q, 1);
                sr = fma(xr, yr, fma(xi, yi, sr));
                si = fma(xi, yr, fma(-xr, yi, si));
            }
        }
        if (r == c) si = 0.0;   // Hermitian: real diagonal
        a[2 * e] = sr;
        a[2 * e + 1] = si;
        fro += sr * sr + si * si;
    }
    fro = sqrt(wave_sum(fro));
    __syncthreads();
    const int kk = k + (k & 1), npairs = kk / 2;
    // off-diagonal entries below this are left alone (they move the largest
    // eigenvalue by far less than a unit of rounding of ||G||^2)
    const double floor_abs = 0x1p-60 * fro;
    for (int sweep = 0; sweep < kMaxSweeps && k > 1; ++sweep) {
        int any_rot = 0;
        for (int rnd = 0; rnd < kk - 1; ++rnd) {
            if (t < npairs) {
                int x = rr_player(t, rnd, kk), y = rr_player(kk - 1 - t, rnd, kk);
                if (x > y) { const int z = x; x = y; y = z; }
                int on = 0;
                if (y < k) {
                    const double app = a[2 * (x * k + x)], aqq = a[2 * (y * k + y)];
                    const double br = a[2 * (y * k + x)], bi = a[2 * (y * k + x) + 1];   // a(x, y)
                    const double ab = hypot(br, bi);
                    if (ab > floor_abs && ab > 0x1p-53 * sqrt(fabs(app * aqq))) {
                        // D = diag(1, e^{-i phi}) makes the pair real; then the
                        // real symmetric Jacobi rotation [[c, s], [-s, c]]
                        const double tau = (aqq - app) / (2.0 * ab);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
                        const double cs = 1.0 / sqrt(fma(tt, tt, 1.0));
                        rot[t][0] = cs;
                        rot[t][1] = tt * cs;
                        rot[t][2] = br / ab;
                        rot[t][3] = bi / ab;
                        on = 1;
                    }
                }
                pa[t] = x;
                pb[t] = y;
                act[t] = on;
            }
            __syncthreads();
            for (int q = 0; q < npairs; ++q) any_rot |= act[q];
            // columns: [a(:, x), a(:, y)] <- [a(:, x), a(:, y)] U,
            // U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
            for (int e = t; e < npairs * k; e += kWave) {
                const int q = e / k, i = e - q * k;
                if (!act[q]) continue;
                const int x = pa[q], y = pb[q];
                const double cs = rot[q][0], sn = rot[q][1], fr = rot[q][2], fi = -rot[q][3];
                const double xr = a[2 * (x * k + i)], xi = a[2 * (x * k + i) + 1];
                double yr = a[2 * (y * k + i)], yi = a[2 * (y * k + i) + 1];
                const double zr = yr * fr - yi * fi, zi = yr * fi + yi * fr;   // e^{-i phi} a(i, y)
                a[2 * (x * k + i)] = cs * xr - sn * zr;
                a[2 * (x * k + i) + 1] = cs * xi - sn * zi;
                a[2 * (y * k + i)] = sn * xr + cs * zr;
                a[2 * (y * k + i) + 1] = sn * xi + cs * zi;
            }
            __syncthreads();
            // rows: [a(x, :); a(y, :)] <- U^* [a(x, :); a(y, :)],
            // U^* = [[c, -s e^{i phi}], [s, c e^{i phi}]]
            for (int e = t; e < npairs * k; e += kWave) {
                const int q = e / k, i = e - q * k;
                if (!act[q]) continue;
                const int x = pa[q], y = pb[q];
                const double cs = rot[q][0], sn = rot[q][1], fr = rot[q][2], fi = rot[q][3];
                const double xr = a[2 * (i * k + x)], xi = a[2 * (i * k + x) + 1];
                const double yr = a[2 * (i * k + y)], yi = a[2 * (i * k + y) + 1];
                const double zr = yr * fr - yi * fi, zi = yr * fi + yi * fr;   // e^{i phi} a(y, i)
                a[2 * (i * k + x)] = cs * xr - sn * zr;
                a[2 * (i * k + x) + 1] = cs * xi - sn * zi;
                a[2 * (i * k + y)] = sn * xr + cs * zr;
                a[2 * (i * k + y) + 1] = sn * xi + cs * zi;
            }
            __syncthreads();
            // the rotated pair is diagonal by construction
            if (t < npairs && act[t]) {
                const int x = pa[t], y = pb[t];
                a[2 * (y * k + x)] = a[2 * (y * k + x) + 1] = 0.0;
                a[2 * (x * k + y)] = a[2 * (x * k + y) + 1] = 0.0;
                a[2 * (x * k + x) + 1] = a[2 * (y * k + y) + 1] = 0.0;
            }
            __syncthreads();
        }
        if (!any_rot) break;
    }
    if (t == 0) {
        double lmax = 0.0;
        for (int i = 0; i < k; ++i) lmax = fmax(lmax, a[2 * (i * k + i)]);
        out[j] = ldexp(sqrt(lmax), ex);
    }
}

}  // namespace

}  // namespace shs

extern "C" int shs_transfer_norm2(int64_t s, int64_t p, int64_t m, const double *G, int64_t ldg, double *norms,
                                  void *stream)
{
    if (s < 0 || s > INT32_MAX) return -1;
    if (p < 0 || p > INT32_MAX / 64) return -2;
    if (m < 1 || m > SHS_MAX_M) return -3;
    if (s == 0) return 0;
    if (p > 0 && !G) return -4;
    if (ldg < (p > 0 ? p : 1)) return -5;
    if (!norms) return -6;
    hipLaunchKernelGGL(shs::gnorm2_kernel, dim3((unsigned)s), dim3(shs::kWave), 0, (hipStream_t)stream, (int)p,
                       (int)m, G, ldg, norms);
    return hipGetLastError() == hipSuccess ? 0 : SHS_ERR_HIP;
}
