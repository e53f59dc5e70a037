// FP64 residual and normwise backward error of a batch of shifted solves.
//
//   Res(:, j m + c) = R(:, c) - (H X_j(:, c) - sigma_j X_j(:, c))
//   eta_j = max_c ||Res(:, jm+c)||_inf / (||H - sigma_j I||_inf ||X_j(:, c)||_inf + ||R(:, c)||_inf)
//
// The product H X over all shifts is one GEMM of the real n x n matrix H
// against the stacked complex solutions (real and imaginary parts are two
// real right-hand sides).  H is m-Hessenberg, so for a block of rows
// [i0, i0 + 64) only columns k >= i0 - m contribute; the kernel starts its
// k loop there and skips the zero band below.  ||H - sigma I||_inf comes
// from the off-diagonal row sums of H computed once at reduction time, so it
// costs O(n) per shift.
#pragma once

#include "common.hpp"

namespace shs {

struct ResidualArgs {
    int n, m, count;            // count = number of listed shifts
    const int32_t *list;        // item -> shift id (nullptr = identity)
    const double *H;            // n x n, ld ldh
    int64_t ldh;
    const double *Rtop;         // m x m, ld m
    const double *shifts;       // per shift id
    const double *X;            // n x (s m) complex, ld ldx
    int64_t ldx;
    double *Res;                // optional, n x (s m) complex, ld ldr (same column layout)
    int64_t ldr;
    unsigned long long *resmax; // per column (s m), max |Res| (bits of a non-negative double)
    unsigned long long *xmax;   // per column, max |X|
};

typedef double shs_dbl4 __attribute__((ext_vector_type(4)));

// The residual on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  A
// workgroup of 4 waves computes 128 rows x 64 complex columns; wave (wr, wc)
// owns rows wr*64 .. +63 and complex columns wc*32 .. +31 as 4 x 4 MFMA
// tiles of 16 x 16.  In LDS the X tile keeps, for each group of 16 complex
// columns, the 16 real parts followed by the 16 imaginary parts, so N-tiles
// 2g and 2g+1 of a wave hold the real and imaginary parts of the same 16
// complex columns and every lane ends with whole complex results.  MFMA
// operand layout: lane l holds A(l%16, l/16) and B(l/16, l%16); result
// register r of lane l is D(4 r + l/16, l%16).
//
// K streams through double-buffered LDS in chunks of 16, stored [row][k]
// with one column of padding (conflict-free fragment reads and stores).
// The chunks k0 .. k0+15 that cover the workgroup's own rows also carry
// X(i, :) for those rows, so sigma X and max |x| are taken from LDS there:
// the epilogue makes no dependent loads.
__global__ __launch_bounds__(256, 2) void residual_mfma_kernel(ResidualArgs a)
{
    constexpr int BM = 128, BNC = 64, BK = 16, PK = BK + 1;
    __shared__ double Hs[2][BM][PK];
    __shared__ double Xs[2][2 * BNC][PK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ncols = a.count * a.m;
    const int n = a.n, m = a.m;
    // The K loop runs downwards from the last row of H: row tiles of one
    // column tile (consecutive workgroups, spread over the XCDs, so each XCD
    // gets long and short K ranges alike) then read the same rows of X at the
    // same time, since all their K ranges end at n.
    const int i0 = blockIdx.x * BM;
    const int w0 = blockIdx.y * BNC;

    shs_dbl4 acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = shs_dbl4{0.0, 0.0, 0.0, 0.0};

    // loads of this thread: H rows i0 + tid%128, k = k0 + tid/128 + 2e (e < 8);
    // X row k0 + tid%16 of complex tile columns tid/16 + 16e (e < 4)
    const double *xcol[4];
    bool xok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int w = w0 + tid / 16 + 16 * e;
        xok[e] = w < ncols;
        const int ww = xok[e] ? w : 0;
        const int item = ww / m, c = ww % m;
        const int sid = a.list ? a.list[item] : item;
        xcol[e] = a.X + ((int64_t)sid * m + c) * a.ldx * 2;
    }
    // this lane's two complex columns (g = 0, 1) and their shifts
    double sgr[2], sgi[2], mx[2] = {0.0, 0.0};
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int w = w0 + wc * 32 + g * 16 + lane % 16;
        const int item = (w < ncols ? w : 0) / m;
        const int sid = a.list ? a.list[item] : item;
        sgr[g] = a.shifts[2 * sid];
        sgi[g] = a.shifts[2 * sid + 1];
    }
    const int hr = tid % BM, hk = tid / BM;
    const int xk = tid % BK, xc = tid / BK;
    double hreg[8], xre[4], xim[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int i = i0 + hr, k = k0 + hk + 2 * e;
            hreg[e] = (i < n && k < n) ? a.H[(int64_t)k * a.ldh + i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + xk;
            const bool ok = xok[e] && k < n;
            xre[e] = ok ? xcol[e][2 * (int64_t)k] : 0.0;
            xim[e] = ok ? xcol[e][2 * (int64_t)k + 1] : 0.0;
        }
    };
    auto lstore = [&](int b) {
#pragma unroll
        for (int e = 0; e < 8; ++e) Hs[b][hr][hk + 2 * e] = hreg[e];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int cc = xc + 16 * e, g = cc / 16, j = cc % 16;
            Xs[b][32 * g + j][xk] = xre[e];
            Xs[b][32 * g + 16 + j][xk] = xim[e];
        }
    };

    int kstart = i0 - m;
    if (kstart < 0) kstart = 0;
    kstart = (kstart / BK) * BK;
    const int ktop = ((n - 1) / BK) * BK;   // chunk holding the last row of H
    gload(ktop);
    lstore(0);
    if (ktop - BK >= kstart) gload(ktop - BK);
    __syncthreads();
    int buf = 0;
    for (int k0 = ktop; k0 >= kstart; k0 -= BK) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[4], bf[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) af[mt] = Hs[buf][wr * 64 + mt * 16 + lane % 16][kk + lane / 16];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bf[nt] = Xs[buf][wc * 64 + nt * 16 + lane % 16][kk + lane / 16];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mt], bf[nt], acc[mt][nt], 0, 0, 0);
        }
        // the chunk holds X(i, :) for the 16 rows i = k0 .. k0+15: block mt of
        // the waves with wr = (k0 - i0) / 64 (uniform per wave)
        const int d = k0 - i0;
        if (d >= 0 && d < BM && (d >> 6) == wr) {
            const int mt = (d & 63) >> 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q != mt) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int kr = 4 * r + lane / 16;   // row k0 + kr
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const double xr = Xs[buf][wc * 64 + 32 * g + lane % 16][kr];
                        const double xi = Xs[buf][wc * 64 + 32 * g + 16 + lane % 16][kr];
                        // H X - sigma X
                        acc[q][2 * g][r] -= sgr[g] * xr - sgi[g] * xi;
                        acc[q][2 * g + 1][r] -= sgr[g] * xi + sgi[g] * xr;
                        const double ax = hypot(xr, xi);
                        mx[g] = (ax > mx[g] || ax != ax) ? ax : mx[g];
                    }
                }
            }
        }
        if (k0 - BK >= kstart) {
            // the other buffer was last read before the previous barrier
            lstore(buf ^ 1);
            if (k0 - 2 * BK >= kstart) gload(k0 - 2 * BK);
        }
        __syncthreads();
        buf ^= 1;
    }

    // epilogue: Res = R - (H X - sigma X) and column maxima
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int w = w0 + wc * 32 + g * 16 + lane % 16;
        double mr = 0.0, mxg = mx[g];
        if (w < ncols) {
            const int item = w / m, c = w % m;
            const int sid = a.list ? a.list[item] : item;
            const int64_t col = (int64_t)sid * m + c;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wr * 64 + mt * 16 + 4 * r + lane / 16;
                    if (i < n) {
                        const double rr = ((i < m) ? a.Rtop[c * m + i] : 0.0) - acc[mt][2 * g][r];
                        const double ri = -acc[mt][2 * g + 1][r];
                        if (a.Res) {
                            double *pr = a.Res + (col * a.ldr + i) * 2;
                            pr[0] = rr;
                            pr[1] = ri;
                        }
                        const double ar = hypot(rr, ri);
                        mr = (ar > mr || ar != ar) ? ar : mr;
                    }
                }
        }
        // lanes l, l+16, l+32, l+48 hold the same column
#pragma unroll
        for (int off = 16; off < 64; off <<= 1) {
            const double orr = __shfl_xor(mr, off), oxx = __shfl_xor(mxg, off);
            mr = (orr > mr || orr != orr) ? orr : mr;
            mxg = (oxx > mxg || oxx != oxx) ? oxx : mxg;
        }
        if (lane < 16 && w < ncols) {
            const int item = w / m, c = w % m;
            const int sid = a.list ? a.list[item] : item;
            const int64_t col = (int64_t)sid * m + c;
            if (mr != mr) mr = __longlong_as_double(0x7ff8000000000000LL);
            if (mxg != mxg) mxg = __longlong_as_double(0x7ff8000000000000LL);
            atomic_max_nonneg(a.resmax + col, mr);
            atomic_max_nonneg(a.xmax + col, mxg);
        }
    }
}

// eta per listed shift; updates status (NaN -> NONFINITE).
__global__ __launch_bounds__(256) void eta_kernel(int n, int m, int count, const int32_t *list,
                                                  const double *shifts, const double *offrow,
                                                  const double *diag, const double *rcolmax,
                                                  const unsigned long long *resmax,
                                                  const unsigned long long *xmax,
                                                  double *eta, int32_t *status)
{
    const int item = blockIdx.x;
    if (item >= count) return;
    const int sid = list ? list[item] : item;
    const double sr = shifts[2 * sid], si = shifts[2 * sid + 1];
    double nh = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = offrow[i] + hypot(diag[i] - sr, si);
        nh = v > nh ? v : nh;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(nh, off);
        nh = o > nh ? o : nh;
    }
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = nh;
    __syncthreads();
    if (threadIdx.x == 0) {
        nh = red[0];
        for (int w = 1; w < 4; ++w) nh = red[w] > nh ? red[w] : nh;
        double e = 0.0;
        bool bad = false;
        for (int c = 0; c < m; ++c) {
            const int64_t col = (int64_t)sid * m + c;
            const double rmx = __longlong_as_double((long long)resmax[col]);
            const double xmx = __longlong_as_double((long long)xmax[col]);
            const double den = nh * xmx + rcolmax[c];
            double v;
            if (rmx != rmx || xmx != xmx) { v = rmx + xmx; bad = true; }
            else v = den > 0.0 ? rmx / den : (rmx > 0.0 ? __longlong_as_double(0x7ff0000000000000LL) : 0.0);
            e = (v > e || v != v) ? v : e;
        }
        eta[sid] = e;
        if (bad && status && status[sid] == 0) status[sid] = 2;
    }
}

// G(:, col) = Ct X(:, col) for the columns of the listed shifts.
// One workgroup per column; rows of Ct are taken 8 at a time.
__global__ __launch_bounds__(256) void g_eval_kernel(int n, int p, int m, int count, const int32_t *list,
                                                     const double *Ct, int64_t ldct,
                                                     const double *X, int64_t ldx,
                                                     double *G, int64_t ldg)
{
    constexpr int PC = 8;
    const int wi = blockIdx.x;            // work column = item * m + c
    const int item = wi / m, c = wi % m;
    if (item >= count) return;
    const int sid = list ? list[item] : item;
    const int64_t col = (int64_t)sid * m + c;
    const double *x = X + col * ldx * 2;
    __shared__ double red[PC * 2][256 / kWave];
    const int tid = threadIdx.x;
    for (int r0 = 0; r0 < p; r0 += PC) {
        double ar[PC], ai[PC];
#pragma unroll
        for (int q = 0; q < PC; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
        for (int i = tid; i < n; i += 256) {
            const double xr = x[2 * (int64_t)i], xi = x[2 * (int64_t)i + 1];
            const double *cc = Ct + (int64_t)i * ldct + r0;
#pragma unroll
            for (int q = 0; q < PC; ++q) {
                if (r0 + q < p) {
                    const double cv = cc[q];
                    ar[q] = fma(cv, xr, ar[q]);
                    ai[q] = fma(cv, xi, ai[q]);
                }
            }
        }
        // wave reduction then across the 4 waves
#pragma unroll
        for (int q = 0; q < PC; ++q) {
            for (int off = 32; off > 0; off >>= 1) {
                ar[q] += __shfl_xor(ar[q], off);
                ai[q] += __shfl_xor(ai[q], off);
            }
        }
        const int wv = tid / kWave;
        if ((tid & 63) == 0) {
#pragma unroll
            for (int q = 0; q < PC; ++q) { red[2 * q][wv] = ar[q]; red[2 * q + 1][wv] = ai[q]; }
        }
        __syncthreads();
        if (tid < 2 * PC) {
            const int q = tid / 2;
            if (r0 + q < p) {
                double sacc = 0.0;
#pragma unroll
                for (int w = 0; w < 256 / kWave; ++w) sacc += red[tid][w];
                G[2 * (col * ldg + r0 + q) + (tid & 1)] = sacc;
            }
        }
        __syncthreads();
    }
}

}  // namespace shs
