// FP64 residual and normwise backward error of a batch of shifted solves.
//
//   Res(:, j m + c) = R(:, c) - (H X_j(:, c) - sigma_j X_j(:, c))
//   eta_j = max_c ||Res(:, jm+c)||_inf / (||H - sigma_j I||_inf ||X_j(:, c)||_inf + ||R(:, c)||_inf)
//
// or, with a dense right-hand side E (nc columns per shift, complex), the same
// with E(:, j nc + c) in place of R(:, c) and its own column maxima.
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
    int n, m, count;            // count = number of listed shifts; m = H's band (H(i, j) = 0 for i > j + m)
    int nc;                     // solution columns per shift (m for [R; 0] right-hand sides)
    const int32_t *list;        // item -> shift id (nullptr = identity)
    const double *H;            // n x n, ld ldh (even, rows n .. ldh-1 zero)
    int64_t ldh;
    const double *Rtop;         // m x m, ld m
    const double *shifts;       // per shift id
    const double *X;            // n x (s m) complex, ld ldx
    int64_t ldx;
    double *Xt;                 // packed copy of the listed columns (residual_pack_kernel)
    int64_t ldxt;               // its row stride: 2 (count m rounded up to 64)
    double *Res;                // optional, n x (s m) complex, ld ldr (same column layout)
    int64_t ldr;
    unsigned long long *resmax; // per column (s m), max |Res| (bits of a non-negative double)
    unsigned long long *xmax;   // per column, max |X|
    const int *dcount;          // if set, the number of listed shifts is read here (count is an upper bound)
    const double *E;            // if set: dense right-hand sides, complex, column sid nc + c at E + col lde * 2
    int64_t lde;
    int ncol_tiles;             // column tiles of residual_mfma_kernel's grid (a multiple of 8)
    unsigned long long *emax;   // with E: per column, max |E|
};

typedef double shs_dbl4 __attribute__((ext_vector_type(4)));

// Xt(k, :) = the listed solutions, row k, k-major: complex column w (item
// w / m, right-hand side w % m) is real column 16 (w / 8) + w % 8 (real part)
// and 8 more (imaginary part), so every 16 real columns hold 8 whole complex
// columns.  Rows n .. and columns past the list are zero.  A tile of 64 rows
// x 32 complex columns goes through LDS (34 KB, four workgroups per CU): its
// loads (along k, the columns of X) are all issued before the LDS stores,
// and it is written along the rows of Xt.
__global__ __launch_bounds__(256) void residual_pack_kernel(ResidualArgs a)
{
    constexpr int TK = 64, TW = 32, PER = TK * TW / 256;   // complex values per thread
    __shared__ double tr[TK][TW + 1], ti[TK][TW + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k0 = blockIdx.x * TK, w0 = blockIdx.y * TW;
    const int m = a.nc;   // columns per shift
    const int ncols = (a.dcount ? *a.dcount : a.count) * m;
    double xr[PER], xi[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int q = wave + 4 * e, w = w0 + q, k = k0 + lane;
        xr[e] = 0.0;
        xi[e] = 0.0;
        if (w < ncols && k < a.n) {
            const int item = w / m, c = w % m;
            const int sid = a.list ? a.list[item] : item;
            const double *x = a.X + (((int64_t)sid * m + c) * a.ldx + k) * 2;
            xr[e] = x[0];
            xi[e] = x[1];
        }
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        tr[lane][wave + 4 * e] = xr[e];
        ti[lane][wave + 4 * e] = xi[e];
    }
    __syncthreads();
    const int rows = (int)residual_pack_rows(a.n);
    for (int e = tid; e < TK * 2 * TW; e += 256) {
        const int kk = e / (2 * TW), j = e % (2 * TW), k = k0 + kk;
        if (k >= rows) break;
        const int q = (j / 16) * 8 + j % 8;   // complex column in the tile
        const double v = (j % 16) < 8 ? tr[kk][q] : ti[kk][q];
        a.Xt[(int64_t)k * a.ldxt + 2 * w0 + j] = v;
    }
}

// LDS of residual_mfma_kernel (dynamic): two stages of a 16-row chunk of
// H^T (128 rows of H) and of Xt (128 real columns).
constexpr int kResidualLds = 2 * 2 * 16 * 128 * (int)sizeof(double);

// The residual on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  A
// workgroup of 4 waves computes 128 rows x 64 complex columns (128 real
// columns of Xt); wave (wr, wc) owns rows wr*64 .. +63 and real columns
// wc*64 .. +63 as 4 x 4 MFMA tiles of 16 x 16.  MFMA operand layout: lane l
// holds A(l%16, l/16) and B(l/16, l%16); result register r of lane l is
// D(4 r + l/16, l%16).  Each 16-column tile holds the real parts of 8
// complex columns and then their imaginary parts, so lanes l and l ^ 8 hold
// the two parts of one complex result.
//
// K streams through two LDS stages that the memory system fills directly
// (global_load_lds_dwordx4, two consecutive doubles of one row of H^T or of
// Xt per lane), k-major on both sides as H and Xt lie in memory; the
// fragment reads of 16 consecutive rows or columns are free of bank
// conflicts.  Rows of H at or past ldh - 1 read row ldh - 2 (never stored);
// chunk rows past n - 1 read column n - 1 of H against zero rows of Xt.
// H is m-Hessenberg, so for a block of rows [i0, i0 + 128) only columns
// k >= i0 - m contribute: the k loop stops there.  It runs downwards from
// the last row of H, so the row tiles of one column tile (consecutive
// workgroups, spread over the XCDs, which then get long and short K ranges
// alike) read the same rows of Xt at the same time.  The chunks that cover
// the workgroup's own rows also carry X(i, :) for those rows, so sigma X and
// max |x| are taken from LDS there: the epilogue makes no dependent loads.
// The grid is 1-D, (n / 128 rounded up) x ncol_tiles workgroups.
__global__ __launch_bounds__(256, 2) void residual_mfma_kernel(ResidualArgs a)
{
    constexpr int BM = 128, BN = 128, BK = 16;
    extern __shared__ double res_smem[];
    auto Hs = reinterpret_cast<double (*)[BK][BM]>(res_smem);
    auto Xs = reinterpret_cast<double (*)[BK][BN]>(res_smem + 2 * BK * BM);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int nc = a.nc;   // columns per shift
    const int ncols = (a.dcount ? *a.dcount : a.count) * nc;
    const int n = a.n, m = a.m;
    // Tile order (1-D grid of ny row tiles x nxp column tiles, nxp the
    // column tiles rounded up to a multiple of 8).  Workgroup L runs on XCD
    // L mod 8.  For the row tiles of group g (8 consecutive row tiles), XCD x
    // takes the column tiles c = (x + g) mod 8, + 8, ...: every XCD gets
    // every row group (whose K ranges differ) and the same number of column
    // tiles in it, and the padding column tiles past the last (which exit
    // at once) rotate over the XCDs from group to group.  On an XCD,
    // consecutive workgroups walk the group's row tiles down one of its
    // column tiles, then the same rows of its next one: the workgroups
    // resident on an XCD share the group's rows of H and each column tile's
    // rows of Xt in its L2.
    int i0, w0;
    {
        const int ny = (n + BM - 1) / BM, ncx = a.ncol_tiles / 8;
        const int L = blockIdx.x, xcd = L & 7, li = L >> 3;
        constexpr int GR = 8;
        const int grp = li / (GR * ncx), r = li - grp * GR * ncx;
        const int rows = min(GR, ny - grp * GR);
        i0 = (grp * GR + r % rows) * BM;
        w0 = ((r / rows) * 8 + ((xcd + grp) & 7)) * (BN / 2);   // first complex column of the tile
    }
    if (w0 >= ncols) return;                // uniform: the tile holds no listed column
    const int q = lane % 16;
    const bool re_lane = q < 8;

    shs_dbl4 acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = shs_dbl4{0.0, 0.0, 0.0, 0.0};

    // this lane's complex column in each N-tile, and its shift
    double sgr[4], sgi[4], mx[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int w = w0 + wc * 32 + nt * 8 + q % 8;
        const int item = (w < ncols ? w : 0) / nc;
        const int sid = a.list ? a.list[item] : item;
        sgr[nt] = a.shifts[2 * sid];
        sgi[nt] = a.shifts[2 * sid + 1];
        mx[nt] = 0.0;
    }
    // wave w moves rows 4w .. 4w+3 of each chunk of both operands
    const double *pa = a.H + min((int64_t)(i0 + 2 * lane), a.ldh - 2);
    const double *pb = a.Xt + 2 * w0 + 2 * lane;
    auto issue = [&](int b, int k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * wave + e;
            const int col = min(k0 + k, n - 1);
            __builtin_amdgcn_global_load_lds((const void *)(pa + (int64_t)col * a.ldh),
                                             (__attribute__((address_space(3))) void *)&Hs[b][k][0], 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(pb + (int64_t)(k0 + k) * a.ldxt),
                                             (__attribute__((address_space(3))) void *)&Xs[b][k][0], 16, 0, 0);
        }
    };

    int kstart = i0 - m;
    if (kstart < 0) kstart = 0;
    kstart = (kstart / BK) * BK;
    const int ktop = ((n - 1) / BK) * BK;   // chunk holding the last row of H
    issue(0, ktop);
    __builtin_amdgcn_s_waitcnt(0x0070);     // vmcnt(0) lgkmcnt(0)
    __syncthreads();
    int b = 0;
    for (int k0 = ktop; k0 >= kstart; k0 -= BK) {
        double af[4][4], bf[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) af[s][mt] = Hs[b][4 * s + lane / 16][wr * 64 + mt * 16 + lane % 16];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bf[s][nt] = Xs[b][4 * s + lane / 16][wc * 64 + nt * 16 + lane % 16];
        }
        // the other stage was last read before the previous barrier
        if (k0 - BK >= kstart) issue(b ^ 1, k0 - BK);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s][mt], bf[s][nt], acc[mt][nt], 0, 0, 0);
        // the chunk holds X(i, :) for the 16 rows i = k0 .. k0+15: block mt of
        // the waves with wr = (k0 - i0) / 64 (uniform per wave)
        const int d = k0 - i0;
        if (d >= 0 && d < BM && (d >> 6) == wr) {
            const int mtd = (d & 63) >> 4;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                if (mt != mtd) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int kr = 4 * r + lane / 16;   // row k0 + kr
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int jj = wc * 64 + nt * 16 + q % 8;
                        const double xr = Xs[b][kr][jj], xi = Xs[b][kr][jj + 8];
                        // H X - sigma X
                        acc[mt][nt][r] -= re_lane ? sgr[nt] * xr - sgi[nt] * xi : sgr[nt] * xi + sgi[nt] * xr;
                        const double ax = hypot(xr, xi);
                        mx[nt] = (ax > mx[nt] || ax != ax) ? ax : mx[nt];
                    }
                }
            }
        }
        // keep the wait for the next chunk behind this chunk's products
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0070);
        __syncthreads();
        b ^= 1;
    }

    // epilogue: Res = R - (H X - sigma X) and column maxima; the real-part
    // lanes (q < 8) take the pair
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int w = w0 + wc * 32 + nt * 8 + q % 8;
        const bool ok = w < ncols;
        const int item = (ok ? w : 0) / nc, c = (ok ? w : 0) % nc;
        const int sid = a.list ? a.list[item] : item;
        const int64_t col = (int64_t)sid * nc + c;
        double mr = 0.0, mxg = mx[nt], me = 0.0;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double v = acc[mt][nt][r], o = __shfl_xor(v, 8);
                const int i = i0 + wr * 64 + mt * 16 + 4 * r + lane / 16;
                if (ok && re_lane && i < n) {
                    double er = (i < m) ? a.Rtop[(c < m ? c : 0) * m + i] : 0.0, ei = 0.0;
                    if (a.E) {
                        const double *pe = a.E + (col * a.lde + i) * 2;
                        er = pe[0];
                        ei = pe[1];
                        const double ae = hypot(er, ei);
                        me = (ae > me || ae != ae) ? ae : me;
                    }
                    const double rr = er - v;
                    const double ri = ei - o;
                    if (a.Res) {
                        double *pr = a.Res + (col * a.ldr + i) * 2;
                        pr[0] = rr;
                        pr[1] = ri;
                    }
                    const double ar = hypot(rr, ri);
                    mr = (ar > mr || ar != ar) ? ar : mr;
                }
            }
        // lanes l, l+16, l+32, l+48 hold the same column
#pragma unroll
        for (int off = 16; off < 64; off <<= 1) {
            const double orr = __shfl_xor(mr, off), oxx = __shfl_xor(mxg, off), oee = __shfl_xor(me, off);
            mr = (orr > mr || orr != orr) ? orr : mr;
            mxg = (oxx > mxg || oxx != oxx) ? oxx : mxg;
            me = (oee > me || oee != oee) ? oee : me;
        }
        if (lane < 8 && ok) {
            if (mr != mr) mr = __longlong_as_double(0x7ff8000000000000LL);
            if (mxg != mxg) mxg = __longlong_as_double(0x7ff8000000000000LL);
            if (me != me) me = __longlong_as_double(0x7ff8000000000000LL);
            atomic_max_nonneg(a.resmax + col, mr);
            atomic_max_nonneg(a.xmax + col, mxg);
            if (a.E) atomic_max_nonneg(a.emax + col, me);
        }
    }
}

// eta per listed shift; updates status (NaN -> NONFINITE).
// m: columns per shift; the right-hand side's column maxima come from
// emax (per column, dense right-hand sides) or rcolmax (per column c of R).
__global__ __launch_bounds__(256) void eta_kernel(int n, int m, int count, const int *dcount, const int32_t *list,
                                                  const double *shifts, const double *offrow,
                                                  const double *diag, const double *rcolmax,
                                                  const unsigned long long *resmax,
                                                  const unsigned long long *xmax,
                                                  const unsigned long long *emax,
                                                  double *eta, int32_t *status)
{
    const int item = blockIdx.x;
    if (item >= (dcount ? *dcount : count)) return;
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
            const double bmx = emax ? __longlong_as_double((long long)emax[col]) : rcolmax[c];
            const double den = nh * xmx + bmx;
            double v;
            if (rmx != rmx || xmx != xmx || bmx != bmx) { v = rmx + xmx + bmx; bad = true; }
            else v = den > 0.0 ? rmx / den : (rmx > 0.0 ? __longlong_as_double(0x7ff0000000000000LL) : 0.0);
            e = (v > e || v != v) ? v : e;
        }
        eta[sid] = e;
        if (bad && status && status[sid] == 0) status[sid] = 2;
    }
}

// G(:, sid m + c) = Ct X(:, sid m + c) for the listed shifts, one
// workgroup per shift.  Rows go in chunks of 256: the chunk's rows of Ct (8
// outputs at a time) are staged in LDS once for the shift's m columns, and
// thread t works on column c = t / TPC (TPC = 256 / m rounded up to a power
// of two) and rows t % TPC, + TPC, ... of the chunk, whose loads of X (the
// threads of one column read consecutive rows) are all issued before they
// are used.  Partial sums are added over the TPC threads of a column in a
// fixed order (shuffles, then the waves in order), so G does not depend on
// scheduling.
__global__ __launch_bounds__(256) void g_eval_kernel(int n, int p, int m, int count, const int32_t *list,
                                                     const double *Ct, int64_t ldct,
                                                     const double *X, int64_t ldx,
                                                     double *G, int64_t ldg)
{
    constexpr int PC = 8, CH = 256, XL = CH / 16;   // rows per chunk; X loads per thread (TPC >= 16)
    const int item = blockIdx.x;
    if (item >= count) return;
    const int sid = list ? list[item] : item;
    int mp = 1;
    while (mp < m) mp *= 2;
    const int tpc = 256 / mp;                 // threads per column
    const int tid = threadIdx.x, c = tid / tpc, r0 = tid % tpc;
    const bool on = c < m;
    const int64_t col = (int64_t)sid * m + (on ? c : 0);
    const double *x = X + col * ldx * 2;
    __shared__ double cts[CH][PC];
    __shared__ double red[4][PC * 2][4];      // per wave: its columns' partial sums
    for (int q0 = 0; q0 < p; q0 += PC) {
        double ar[PC], ai[PC];
#pragma unroll
        for (int q = 0; q < PC; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
        for (int i0 = 0; i0 < n; i0 += CH) {
            __syncthreads();                  // the previous chunk is read
            for (int e = tid; e < CH * PC; e += 256) {
                const int i = i0 + e / PC, q = e % PC;
                cts[e / PC][q] = (i < n && q0 + q < p) ? Ct[(int64_t)i * ldct + q0 + q] : 0.0;
            }
            double xr[XL], xi[XL];
#pragma unroll
            for (int l = 0; l < XL; ++l) {
                const int ii = r0 + l * tpc, i = i0 + ii;
                const bool ok = on && ii < CH && i < n;
                xr[l] = ok ? x[2 * (int64_t)i] : 0.0;
                xi[l] = ok ? x[2 * (int64_t)i + 1] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int l = 0; l < XL; ++l) {
                const int ii = r0 + l * tpc;
                if (ii < CH) {
#pragma unroll
                    for (int q = 0; q < PC; ++q) {
                        const double cv = cts[ii][q];
                        ar[q] = fma(cv, xr[l], ar[q]);
                        ai[q] = fma(cv, xi[l], ai[q]);
                    }
                }
            }
        }
        // sum over the lanes of one column inside the wave (tpc >= 16)
        const int span = tpc < kWave ? tpc : kWave;
#pragma unroll
        for (int q = 0; q < PC; ++q) {
            for (int off = 1; off < span; off <<= 1) {
                ar[q] += __shfl_xor(ar[q], off);
                ai[q] += __shfl_xor(ai[q], off);
            }
        }
        const int wv = tid / kWave, lane = tid % kWave;
        // lane 0 of each column's span in this wave holds its partial sums
        if (lane % span == 0) {
            const int slot = lane / span;     // column slot inside the wave (< 64 / span <= 4)
#pragma unroll
            for (int q = 0; q < PC; ++q) { red[wv][2 * q][slot] = ar[q]; red[wv][2 * q + 1][slot] = ai[q]; }
        }
        __syncthreads();
        // one thread per (column, output): add the waves that hold the column, in order
        if (tid < m * 2 * PC) {
            const int cc = tid / (2 * PC), e = tid % (2 * PC), q = e / 2;
            if (q0 + q < p) {
                const int t0 = cc * tpc;                  // first thread of column cc
                const int w0 = t0 / kWave, nw = (tpc + kWave - 1) / kWave;
                double sacc = 0.0;
                for (int w = w0; w < w0 + nw; ++w) {
                    const int slot = (t0 % kWave) / span;
                    sacc += red[w][e][slot];
                }
                G[2 * (((int64_t)sid * m + cc) * ldg + q0 + q) + (e & 1)] = sacc;
            }
        }
        __syncthreads();
    }
}

}  // namespace shs
