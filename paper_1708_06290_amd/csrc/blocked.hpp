// Blocked FP64 sweep: Step 2 of Section 3.1 done once per row tile for all
// shifts together, as the paper's "Step 2, revisited" does per block.
//
// The per-shift sweep (sweep.hpp) walks every row above a pivot through every
// reflector.  Grouping the n_b = 64 R steps of one row tile (rows lo .. hi-1)
// into one block transform P_blk = P_{hi-1} ... P_lo (of size n_b + m, acting
// on window columns lo-m .. hi-1) changes the update of every row i < lo into
//
//   z_i <- [ H(i, lo-m .. hi-1-m)  z_i ] * M_blk,      M_blk = P_blk(:, 0:m),
//
// where z_i (m complex values) are row i's carried window columns: before
// the tile they are columns hi-m .. hi-1, after it columns lo-m .. lo-1.  The
// first n_b rows of M_blk (M1) multiply the fresh columns of H, which are
// real and the same for every shift; the last m rows (M2) multiply z_i.  So
// the update of all rows above the tile, for all shifts, is ONE real GEMM
// H(0:lo, lo-m : hi-m) * [Re M1 | Im M1 for every shift] on the FP64 matrix
// cores, plus a per-shift (2m x 2m) product with z.  The shift enters only
// through the diagonal entries H(i, i) - sigma of the m rows i = lo-m .. lo-1,
// whose diagonal lies in the block: those rows get -sigma M1(i - lo + m, :).
//
// Per row tile, bottom to top:
//   blk_tri_kernel  one wavefront per shift: loads the tile's window (carried
//                   columns from Z, fresh columns from H), produces the tile's
//                   reflectors with the same code as the per-shift sweep
//                   (stored for the Q* pass), then forms M_blk by applying
//                   them to [I_m; 0] (lanes c < m, one column each, a sliding
//                   (m+1)-row window; where mblk_groups allows, two or four
//                   lane groups run a share of the steps each and their rows
//                   are combined afterwards) and writes it real-ified for
//                   the GEMM.
//   zupd_kernel     the GEMM above, in place on Z.
// The top tile's kernel ends with the m x m back substitution, as before.
//
// Above the bottom tile the updates are grouped by D tiles a_1, a_2, ...
// (bottom to top): after a_k (k < D) only the next tile's rows get the
// group's composite transform so far (they are needed next); after a_D,
// every row above gets all D at once.  For two tiles a, b = a - 1,
//
//   z <- H(:, fresh_b) M1_b + H(:, fresh_a) (M1_a M2_b) + z (M2_a M2_b),
//
// one GEMM over the contiguous columns fresh_b, fresh_a; in general K = k n_b
// after a_k.  The composite's operand rows sit at the end of Bm, newest tile
// first (so it lines up with H's columns): a_k writes M1 to rows
// (D-k) n_b .. (D-k+1) n_b - 1 and multiplies the older rows below them by
// its M2 in place, and the composite carried matrix M2_{a_1} ... M2_{a_k} is
// formed alongside.  This divides the passes over Z by D and multiplies K
// per update launch by D.
//
// Z holds, for work item (shift) w, the carried columns of every row as 2m
// real columns w W .. w W + 2m - 1 (real parts, then imaginary parts) of a
// column-major n x (W items) array; W, the per-shift column stride, is 2m
// (4m with a dense right-hand side) rounded up to a power of two (>= 2), or
// to 24 or 48 (blk_cols), so a 16-column MFMA block holds one shift
// (W = 16), part of one (W = 32, 48, 64), several whole ones (W < 16), or
// the end of one shift and the start of the next (W = 24).  The main
// product never mixes columns; the carried part of W < 16 and W = 24 does,
// with zero weights (see zupd_kernel).
// The bottom tile's carried columns are
// plain columns of H - sigma I, so its GEMM folds them into K (K = n_b + m)
// and reads no Z.
#pragma once

#include "sweep.hpp"
#include "kernels.hpp"

namespace shs {

__host__ __device__ constexpr int blk_width(int m)
{
    return m <= 1 ? 2 : (m <= 2 ? 4 : (m <= 4 ? 8 : (m <= 8 ? 16 : (m <= 16 ? 32 : 64))));
}

// Real columns per shift of the carried-column array: 2m for the carried
// columns z, and with a dense right-hand side 2m more for e (its m columns'
// real parts, then imaginary parts), rounded up to a power of two, 24 or 48.
// 24 and 48 (for 17 .. 24 and 33 .. 48 active columns) keep a quarter of
// the update from being spent on padding; a 16-column block then holds
// columns of at most two shifts (24) or of one (48).
__host__ __device__ constexpr int blk_cols(int m, bool dense)
{
    const int aw = dense ? 4 * m : 2 * m;
    return aw > 32 && aw <= 48 ? 48 : (aw > 16 && aw <= 24 ? 24 : blk_width(dense ? 2 * m : m));
}

// The block-transform chain of the tile kernel is split over lane groups up
// to these m (see blk_tri_kernel; with a dense right-hand side beyond m = 8
// the group windows would push the kernel's LDS past what keeps its
// occupancy): 4 groups where the lanes and the reflector chunk (cs steps of
// m+1-step phase groups) allow it, else 2, else 1 (no split).
constexpr int kMblkSplitMaxM = 16;
constexpr int kMblkSplitMaxMDense = 8;
template <int M, bool DENSE>
__host__ __device__ constexpr int mblk_groups(int np, int cs)
{
    const int lg = DENSE ? 2 * M : M;
    if (M > (DENSE ? kMblkSplitMaxMDense : kMblkSplitMaxM)) return 1;
    if (4 * lg <= kWave && cs >= 4 * np) return 4;
    if (2 * lg <= kWave && cs >= 2 * np) return 2;
    return 1;
}

// Columns of one tile of the update GEMM: 128, or 96 for 24- and 48-column
// shifts.  Either way a tile, and each half of it, holds whole shifts.  That
// is what lets the update run in place: the carried part of a shift reads
// all of the shift's columns, and no other workgroup writes them.
__host__ __device__ constexpr int zupd_bn(int w) { return w == 24 || w == 48 ? 96 : 128; }

template <typename T>
struct BlkTriArgsT {
    int n;
    int count;                 // work items (= launched workgroups)
    int t, ntiles;             // this row tile, number of row tiles
    const T *H;
    int64_t ldh;
    const double *shifts;      // interleaved complex, by shift id
    const int32_t *list;       // work item -> shift id (nullptr = identity)
    const double *Rtop;        // m x m upper triangle of R (ld m)
    T *refl;                   // per shift id reflector store
    int64_t refl_stride;
    T *Y;                      // per shift id: m x m complex, or n x m with a dense right-hand side
    int64_t y_stride;
    int32_t *status;           // per shift id
    const T *Z;                // carried columns (see above), ld ldz
    int64_t ldz;
    T *Bm;                     // M1 (and for the bottom tile M2) rows, row-major: row k at Bm + k ldb
    int64_t ldb;               // row stride of Bm (columns of Z, a multiple of 128)
    T *M2;                     // per work item W x W real (row-major): written by a dense bottom tile
    const T *M2p;              // per work item W x W: composite M2 of the group so far (k >= 2)
    T *M2q;                    // per work item W x W: composite M2 including this tile
    int gk;                    // 0: bottom tile; k = 1 .. D: k-th tile of a group
    int D;                     // tiles per group; Bm holds D TT + m rows
    const int *dcount;         // if set, the number of work items is read here (count is an upper bound)
};
using BlkTriArgs = BlkTriArgsT<double>;

// Block-transform destinations (n_b = TT rows of M1 per tile):
//   bottom        Bm rows 0 .. n_b+m-1 (M1 and M2, K = n_b + m)
//   k-th of group M1 -> Bm rows (D-k) TT .. (D-k+1) TT - 1; rows below it,
//                 up to D TT - 1, <- themselves times M2; M2q <- M2p M2
//
// With a dense right-hand side (DENSE: e_i, m complex values per row, in Z
// after the carried columns) the rows above the tile also need
// e_i -= sum_k R_sigma(i, k) y_k over the tile's steps k.  R_sigma(i, k) is
// the column that leaves the window at step k, a linear function of the
// row's window before the tile, so the sum is [H(i, fresh) z_i] N_blk with
// N_blk = sum_k P_{hi-1} ... P_k e_k y_k (e_k the unit vector of window
// column k), which the recursion v <- P_k (v + e_k y_k), k = lo .. hi-1,
// forms next to M_blk: the same sliding window, with y_k entering where M_blk
// lets a zero row in.  The GEMM operand of a shift becomes [M1 | -N1] and
// the carried matrix [[M2, -N2], [0, I]], which maps [z e] to
// [z M2, e - z N2]; the bottom tile folds M2 and -N2 into K and carries e
// through the identity.
// Rows per lane of the tile kernels: the per-shift sweep's choice in FP64;
// in FP32 at most 4 (with 8 the step body unrolled per row slot no longer fits
// the registers and spills up to a kilobyte per lane).
template <typename T, int M, bool DENSE>
__host__ __device__ constexpr int blk_rb()
{
    constexpr int r = rows_per_lane<T, M, DENSE>();
    return sizeof(T) == 4 && r > 4 ? 4 : r;
}

template <typename T, int M, bool DENSE>
__global__ __launch_bounds__(64, 2) void blk_tri_kernel(BlkTriArgsT<T> a)
{
    constexpr int RB = blk_rb<T, M, DENSE>();
    using Sh = SweepShape<T, M, DENSE, RB>;
    constexpr int R = Sh::R, TT = Sh::TT, S = Sh::S, NP = Sh::NP, EM = Sh::EM;
    constexpr int W = blk_cols(M, DENSE);
    constexpr int AW = DENSE ? 4 * M : 2 * M;   // active real columns per shift
    constexpr int NL = DENSE ? 2 * M : M;       // lanes forming the block transform
    __shared__ T lds_rs[2 * M * M];
    __shared__ T lds_m2[W * W];   // the carried matrix of this tile, real form
    const int item = blockIdx.x;
    if (item >= (a.dcount ? *a.dcount : a.count)) return;
    const int sid = a.list ? a.list[item] : item;
    const int lane = threadIdx.x;
    const int n = a.n, t = a.t;
    const int lo = t * TT, hi = min(n, lo + TT);
    const bool bottom = t == a.ntiles - 1;
    const T sgr = (T)a.shifts[2 * sid], sgi = (T)a.shifts[2 * sid + 1];
    T *rf = a.refl + (int64_t)sid * a.refl_stride;
    T *Y = a.Y + (int64_t)sid * a.y_stride;
    const int64_t tstride = refl_tile_stride<T>(TT, S);
    const T *H = a.H;
    const int64_t ldh = a.ldh;

    // ---- window at step hi-1: slot p holds position j = (p - (hi-1)) mod (m+1),
    // column hi-1-m+j.  Position 0 is the fresh column hi-1-m (from H); the
    // others are the carried columns hi-m .. hi-1 (from Z, or from H for the
    // bottom tile).  Rows past n only exist in the bottom tile.
    T wr[R][NP], wi[R][NP], er[R][EM], ei[R][EM];
    {
        const int q0 = (hi - 1) % NP;
        const T *Zi = a.Z + (int64_t)item * W * a.ldz;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int j = (p - q0 + NP) % NP;
            const int col = hi - 1 - M + j;
            if (bottom || j == 0) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = lo + r * kWave + lane;
                    const T v = (col >= 0 && i < n) ? H[(int64_t)col * ldh + i] : T(0);
                    const bool dg = i == col;
                    wr[r][p] = dg ? v - sgr : v;
                    wi[r][p] = dg ? -sgi : T(0);
                }
            } else {
                const T *zr = Zi + (int64_t)(j - 1) * a.ldz;
                const T *zi = Zi + (int64_t)(M + j - 1) * a.ldz;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = lo + r * kWave + lane;
                    wr[r][p] = zr[i];
                    wi[r][p] = zi[i];
                }
            }
        }
        if constexpr (DENSE) {
            // the tile's rows of the right-hand side, after every tile below
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const T *pr = Zi + (int64_t)(2 * M + c) * a.ldz;
                const T *pi = Zi + (int64_t)(3 * M + c) * a.ldz;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = lo + r * kWave + lane;
                    er[r][c] = i < n ? pr[i] : T(0);
                    ei[r][c] = i < n ? pi[i] : T(0);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) { er[r][0] = T(0); ei[r][0] = T(0); }
        }
    }

    bool singular = false, nonfinite = false;
    tri_phase<T, M, DENSE, true, RB>(n, lo, hi, lane, H, ldh, sgr, sgi, rf, tstride, Y, lds_rs, wr, wi, er, ei,
                                     singular, nonfinite);
    // the tile's reflector stores complete before they are read back below
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");

    if (t == 0) {
        // earlier tiles recorded a singular step in the status word
        const bool before = !bottom && a.status[sid] == 1;
        if constexpr (DENSE) nonfinite = __any(nonfinite);
        finish_shift<T, M, DENSE>(n, lane, a.Rtop, Y, lds_rs, a.status + sid, singular || before, nonfinite);
        return;
    }
    if (lane == 0 && (bottom || singular)) a.status[sid] = singular ? 1 : 0;

    // ---- M_blk = P_{hi-1} ... P_lo [I_m; 0]: lane c < m owns column c ----------
    // (where mblk_groups allows, the steps are split over lane groups, below)
    // P_k acts on rows k-lo .. k-lo+m of M_blk.  Applied from P_lo upwards, row
    // p is final once P_{lo+p} is done, so each lane keeps a window of m+1
    // rows (row p in slot p mod (m+1)), emits the finished row and lets the
    // next (zero) row in.  With a dense right-hand side, lane m + c forms
    // column c of N_blk the same way, y_k(c) entering at row k-lo+m before
    // P_k.  The tile's reflectors come back through LDS in chunks of CS steps
    // that the whole wave loads (coalesced, the next chunk in flight while
    // the current one is used), so the serial chain never waits on memory.
    {
        // steps per chunk: whole phase groups, about 12 elements per lane
        constexpr int CS = NP * ((12 * kWave / S) / NP > 0 ? (12 * kWave / S) / NP : 1);
        constexpr int CE = CS * S;                          // elements per chunk
        constexpr int PL = (CE + kWave - 1) / kWave;
        __shared__ T lds_ch[CE];
        T pre[PL];
        const bool isn = DENSE && lane >= M && lane < 2 * M;   // an N_blk column
        const int c = lane < NL ? (isn ? lane - M : lane) : 0;
        const int nb = hi - lo;
        const int K = bottom ? nb + M : nb;
        const int boff = a.gk >= 1 ? (a.D - a.gk) * TT : 0;
        // row p of the block transform is row boff + p of Bm; this column's
        // real and imaginary parts are the shift's columns cre and cre + m
        const int cre = isn ? 2 * M + c : c;
        T *bcr = a.Bm + (int64_t)boff * a.ldb + item * W + cre;
        T *bci = bcr + M;
        // the carried matrix is assembled in LDS: z rows times M2 and -N2, the
        // identity for e
        for (int e = lane; e < W * W; e += kWave) {
            const int rr = e / W, cc = e % W;
            lds_m2[e] = (DENSE && rr == cc && rr >= 2 * M && rr < 4 * M) ? T(1) : T(0);
        }
        // slots past hi - 1 are loaded from a clamped address and never used
        auto fetch = [&](int cb) {
#pragma unroll
            for (int e = 0; e < PL; ++e) {
                const int idx0 = e * kWave + lane;
                const int idx = idx0 < CE ? idx0 : CE - 1;
                const int ks = idx / S, el = idx - ks * S;
                const int k = min(cb + ks, hi - 1);
                pre[e] = refl_slot<T>(rf, k, TT, tstride, S)[el];
            }
        };
        // a shift with a non-finite sigma gets a zero transform: its own
        // result is flagged by its status, and its Z columns stay finite
        const bool bad = !isfinite(sgr) || !isfinite(sgi);
        const T sgn = isn ? T(-1) : T(1);   // the operand holds -N_blk
        auto emit = [&](int p, T xr, T xi) {
            if (bad) xr = xi = T(0);
            xr *= sgn;
            xi *= sgn;
            if (p < K) {
                bcr[(int64_t)p * a.ldb] = xr;
                bci[(int64_t)p * a.ldb] = xi;
            } else {
                // real form of z times the m x m block: [zr zi] [[Re, Im], [-Im, Re]]
                const int cp = p - nb;
                lds_m2[cp * W + cre] = xr;
                lds_m2[cp * W + M + cre] = xi;
                lds_m2[(M + cp) * W + cre] = -xi;
                lds_m2[(M + cp) * W + M + cre] = xr;
            }
        };
        constexpr int G = mblk_groups<M, DENSE>(NP, CS);
        if constexpr (G < 2) {
            T ur[NP], ui[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) { ur[p] = (!isn && p == c) ? T(1) : T(0); ui[p] = T(0); }
            fetch(lo);
            for (int cb = lo; cb < hi; cb += CS) {
                // one wave per workgroup: its LDS operations complete in order,
                // so the chunk can overwrite the previous one in place
#pragma unroll
                for (int e = 0; e < PL; ++e) {
                    const int idx = e * kWave + lane;
                    if (idx < CE) lds_ch[idx] = pre[e];
                }
                if (cb + CS < hi) fetch(cb + CS);
                if (lane < NL) {
                const int ce = min(hi, cb + CS);
                for (int kb = cb; kb < ce; kb += NP) {
                static_for<NP>([&](auto sc) {
                    constexpr int st = decltype(sc)::value;
                    const int k = kb + st;
                    if (k < ce) {
                        const T *pv = lds_ch + (k - cb) * S;
                        const T tau = pv[0];
                        T vr[M], vi[M];
#pragma unroll
                        for (int j = 0; j < M; ++j) { vr[j] = pv[2 + 2 * j]; vi[j] = pv[3 + 2 * j]; }
                        if constexpr (DENSE) {
                            // y_k(c) enters at window position m (row k-lo+m)
                            if (isn) {
                                ur[(st + M) % NP] += pv[2 + 2 * M + 2 * c];
                                ui[(st + M) % NP] += pv[3 + 2 * M + 2 * c];
                            }
                        }
                        // s = v^* u over positions j = 0 .. m (v_m = 1); position j in slot (st + j) mod (m+1)
                        T sr = ur[(st + M) % NP], si = ui[(st + M) % NP];
#pragma unroll
                        for (int j = 0; j < M; ++j) {
                            const int q = (st + j) % NP;
                            sr = fma(vr[j], ur[q], fma(vi[j], ui[q], sr));
                            si = fma(vr[j], ui[q], fma(-vi[j], ur[q], si));
                        }
                        const T tr = tau * sr, ti = tau * si;
#pragma unroll
                        for (int j = 0; j < M; ++j) {
                            const int q = (st + j) % NP;
                            ur[q] = fma(-vr[j], tr, fma(vi[j], ti, ur[q]));
                            ui[q] = fma(-vr[j], ti, fma(-vi[j], tr, ui[q]));
                        }
                        ur[(st + M) % NP] -= tr;
                        ui[(st + M) % NP] -= ti;
                        emit(k - lo, ur[st], ui[st]);
                        ur[st] = T(0);
                        ui[st] = T(0);
                    }
                });
                }
                }
            }
            // rows nb .. nb+m-1 are still in the window (row nb+m is the zero row)
            if (lane < NL) {
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const int p = nb + ((q - nb % NP) + NP) % NP;
                    if (p < nb + M) emit(p, ur[q], ui[q]);
                }
            }
        } else {
            // The chain split over G lane groups.  Group g (lanes g L .. g L +
            // L-1, L = m, or 2m with a dense right-hand side: the M_blk
            // columns, then the N_blk ones) runs steps g h .. g h + h_g - 1 of
            // the tile (h a whole number of phase groups) from the identity
            // window (M_blk columns) or the zero one (N_blk columns), so it
            // forms E_g and EN_g, the rows those steps finish, and F_g and
            // NF_g, its final windows.  The steps are linear in the window
            // (affine for N_blk, whose y_k enter), so with the true windows at
            // the start of group g, W_g = F_{g-1} W_{g-1} (W_0 = I) and Nw_g =
            // F_{g-1} Nw_{g-1} + NF_{g-1} (Nw_0 = 0), group g's true rows are
            // E_g W_g and E_g Nw_g + EN_g, and the rows nb .. nb+m-1 left in
            // the window after the last step are W_G and Nw_G.
            constexpr int LG = DENSE ? 2 * M : M;
            constexpr int NW = DENSE ? 2 : 1;                     // windows per group
            constexpr int CSg = NP * (CS / (G * NP));            // steps per chunk and group
            static_assert(CSg >= NP && G * CSg * S <= CE && G * LG <= kWave, "chunk");
            static_assert(2 * NW * G * M * M <= CE, "F in the chunk buffer");
            // W_1 .. W_G (and Nw_1 .. Nw_G), complex, row-major
            __shared__ T lds_w[2 * NW * G * M * M];
            const int hq = NP * ((nb + G * NP - 1) / (G * NP)); // steps per group, whole phase groups
            const int g = lane / LG, jl = lane % LG;
            const bool gisn = DENSE && jl >= M;                  // an N_blk column
            const int cg = gisn ? jl - M : jl;
            const bool act = lane < G * LG;
            const int gs = g * hq;
            const int hg = act ? max(0, min(hq, nb - gs)) : 0;
            T *gcr = a.Bm + (int64_t)boff * a.ldb + item * W + (gisn ? 2 * M : 0) + cg;
            const T gsgn = gisn ? T(-1) : T(1);                  // the operand holds -N_blk
            // raw rows straight into Bm (group 0's are final), zero for a bad shift
            auto emit_raw = [&](int pr, T xr, T xi) {
                if (bad) xr = xi = T(0);
                gcr[(int64_t)pr * a.ldb] = gsgn * xr;
                gcr[(int64_t)pr * a.ldb + M] = gsgn * xi;
            };
            // chunk of CSg steps of every group, loaded by the whole wave;
            // steps past the tile read a clamped slot and are not used
            auto fetch_g = [&](int j0) {
#pragma unroll
                for (int e = 0; e < PL; ++e) {
                    const int idx0 = e * kWave + lane;
                    const int idx = idx0 < G * CSg * S ? idx0 : G * CSg * S - 1;
                    const int grp = idx / (CSg * S), rem = idx - grp * (CSg * S);
                    const int ks = rem / S, el = rem - ks * S;
                    const int k = lo + min(grp * hq + j0 + ks, nb - 1);
                    pre[e] = refl_slot<T>(rf, k, TT, tstride, S)[el];
                }
            };
            T ur[NP], ui[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) { ur[p] = (act && !gisn && p == cg) ? T(1) : T(0); ui[p] = T(0); }
            fetch_g(0);
            for (int j0 = 0; j0 < hq; j0 += CSg) {
                // one wave: the previous chunk's LDS reads are complete
#pragma unroll
                for (int e = 0; e < PL; ++e) {
                    const int idx = e * kWave + lane;
                    if (idx < G * CSg * S) lds_ch[idx] = pre[e];
                }
                if (j0 + CSg < hq) fetch_g(j0 + CSg);
                for (int kb = 0; kb < CSg; kb += NP) {
                    static_for<NP>([&](auto sc) {
                        constexpr int st = decltype(sc)::value;
                        const int kk = j0 + kb + st;   // step within the group, kk = st (mod m+1)
                        if (kk < hg) {
                            const T *pv = lds_ch + (g * CSg + kb + st) * S;
                            const T tau = pv[0];
                            T vr[M], vi[M];
#pragma unroll
                            for (int j = 0; j < M; ++j) { vr[j] = pv[2 + 2 * j]; vi[j] = pv[3 + 2 * j]; }
                            if constexpr (DENSE) {
                                // y_k(c) enters at window position m (row k-lo+m)
                                if (gisn) {
                                    ur[(st + M) % NP] += pv[2 + 2 * M + 2 * cg];
                                    ui[(st + M) % NP] += pv[3 + 2 * M + 2 * cg];
                                }
                            }
                            T sr = ur[(st + M) % NP], si = ui[(st + M) % NP];
#pragma unroll
                            for (int j = 0; j < M; ++j) {
                                const int q = (st + j) % NP;
                                sr = fma(vr[j], ur[q], fma(vi[j], ui[q], sr));
                                si = fma(vr[j], ui[q], fma(-vi[j], ur[q], si));
                            }
                            const T tr = tau * sr, ti = tau * si;
#pragma unroll
                            for (int j = 0; j < M; ++j) {
                                const int q = (st + j) % NP;
                                ur[q] = fma(-vr[j], tr, fma(vi[j], ti, ur[q]));
                                ui[q] = fma(-vr[j], ti, fma(-vi[j], tr, ui[q]));
                            }
                            ur[(st + M) % NP] -= tr;
                            ui[(st + M) % NP] -= ti;
                            emit_raw(gs + kk, ur[st], ui[st]);
                            ur[st] = T(0);
                            ui[st] = T(0);
                        }
                    });
                }
            }
            // F_g and NF_g (row i = window row hg + i, in slot (hg + i) mod
            // (m+1)) into the chunk buffer, complex, row-major per group
            T *lf = lds_ch;
            auto fidx = [&](int kind, int gg, int i, int cc) { return 2 * (((kind * G + gg) * M + i) * M + cc); };
            if (act) {
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const int i = ((q - hg) % NP + NP) % NP;
                    if (i < M) {
                        lf[fidx(gisn ? 1 : 0, g, i, cg)] = ur[q];
                        lf[fidx(gisn ? 1 : 0, g, i, cg) + 1] = ui[q];
                    }
                }
            }
            // W_1 = F_0, W_{g+1} = F_g W_g, and Nw_1 = NF_0, Nw_{g+1} = F_g Nw_g
            // + NF_g (lds_w slot g-1 holds W_g, Nw_g); one wave, so each
            // product reads the previous one's stores
            for (int e = lane; e < NW * M * M; e += kWave) {
                const int kind = e / (M * M), r = e % (M * M);
                const int s0 = fidx(kind, 0, 0, 0) + 2 * r;
                lds_w[s0] = lf[s0];
                lds_w[s0 + 1] = lf[s0 + 1];
            }
            for (int gg = 1; gg < G; ++gg) {
                for (int e = lane; e < NW * M * M; e += kWave) {
                    const int kind = e / (M * M), r = e % (M * M), i = r / M, cc = r % M;
                    const T *fr = lf + fidx(0, gg, i, 0);
                    T xr = T(0), xi = T(0);
                    if (kind == 1) {
                        xr = lf[fidx(1, gg, i, cc)];
                        xi = lf[fidx(1, gg, i, cc) + 1];
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const T ar = fr[2 * q], ai = fr[2 * q + 1];
                        const T br = lds_w[fidx(kind, gg - 1, q, cc)], bi = lds_w[fidx(kind, gg - 1, q, cc) + 1];
                        xr = fma(ar, br, fma(-ai, bi, xr));
                        xi = fma(ar, bi, fma(ai, br, xi));
                    }
                    lds_w[fidx(kind, gg, i, cc)] = xr;
                    lds_w[fidx(kind, gg, i, cc) + 1] = xi;
                }
            }
            // the raw rows of groups 1 .. G-1 (written above by other lanes)
            // become E_g W_g (and -(E_g Nw_g + EN_g): the raw N_blk rows are
            // stored negated)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            T *brow = a.Bm + (int64_t)boff * a.ldb + item * W;
            for (int pr = hq + lane; pr < nb; pr += kWave) {
                const int gg = pr / hq;
                T *row = brow + (int64_t)pr * a.ldb;
                T er[M], ei[M];
#pragma unroll
                for (int q = 0; q < M; ++q) { er[q] = row[q]; ei[q] = row[M + q]; }
#pragma unroll
                for (int kind = 0; kind < NW; ++kind) {
#pragma unroll
                    for (int cc = 0; cc < M; ++cc) {
                        T xr = T(0), xi = T(0);
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            const T br = lds_w[fidx(kind, gg - 1, q, cc)], bi = lds_w[fidx(kind, gg - 1, q, cc) + 1];
                            xr = fma(er[q], br, fma(-ei[q], bi, xr));
                            xi = fma(er[q], bi, fma(ei[q], br, xi));
                        }
                        if (kind == 0) {
                            row[cc] = bad ? T(0) : xr;
                            row[M + cc] = bad ? T(0) : xi;
                        } else {
                            row[2 * M + cc] = bad ? T(0) : row[2 * M + cc] - xr;
                            row[3 * M + cc] = bad ? T(0) : row[3 * M + cc] - xi;
                        }
                    }
                }
            }
            // rows nb .. nb+m-1: W_G and Nw_G (into K for the bottom tile,
            // else the carried matrix in its real form)
            for (int e = lane; e < NW * M * M; e += kWave) {
                const int kind = e / (M * M), r = e % (M * M), i = r / M, cc = r % M;
                const T s = kind ? T(-1) : T(1);
                T xr = s * lds_w[fidx(kind, G - 1, i, cc)], xi = s * lds_w[fidx(kind, G - 1, i, cc) + 1];
                if (bad) xr = xi = T(0);
                const int cre = kind * 2 * M + cc;
                if (nb + i < K) {
                    brow[(int64_t)(nb + i) * a.ldb + cre] = xr;
                    brow[(int64_t)(nb + i) * a.ldb + M + cre] = xi;
                } else {
                    lds_m2[i * W + cre] = xr;
                    lds_m2[i * W + M + cre] = xi;
                    lds_m2[(M + i) * W + cre] = -xi;
                    lds_m2[(M + i) * W + M + cre] = xr;
                }
            }
        }
        // one wave: its LDS writes above are complete before these reads
        if (DENSE && bottom) {
            // the bottom tile's operand covers z through K; e goes through
            T *pm = a.M2 + (int64_t)item * W * W;
            for (int e = lane; e < W * W; e += kWave) pm[e] = lds_m2[e];
        }
        if (a.gk == 1) {
            T *pm = a.M2q + (int64_t)item * W * W;
            for (int e = lane; e < W * W; e += kWave) pm[e] = lds_m2[e];
        }
        if (a.gk >= 2) {
            // the older composite rows: B <- B M2 (real form)
            const int r1 = (a.D - a.gk + 1) * TT, nrows = (a.gk - 1) * TT;
            T *bb = a.Bm + (int64_t)r1 * a.ldb + item * W;
            // each lane one row at a time: the whole row first (its loads in
            // flight together; up to 16 active columns the next row's are
            // issued before this one is multiplied, beyond that the registers
            // are short), then the product with M2 from LDS; the opaque
            // offset keeps the compiler from hoisting all the LDS reads out
            // of the row loop into registers
            constexpr bool PF = AW <= 16;
            // output columns per pass: all of them up to 32, else 16 at a
            // time (the row itself stays in registers)
            constexpr int QC = AW > 32 ? 16 : AW;
            T o[AW];
            if (PF && lane < nrows) {
#pragma unroll
                for (int q = 0; q < AW; ++q) o[q] = bb[(int64_t)lane * a.ldb + q];
            }
#pragma unroll 1
            for (int p = lane; p < nrows; p += kWave) {
                T *row = bb + (int64_t)p * a.ldb;
                T on[PF ? AW : 1];
                const int pn = p + kWave < nrows ? p + kWave : p;
#pragma unroll
                for (int q = 0; q < AW; ++q) {
                    if constexpr (PF) on[q] = bb[(int64_t)pn * a.ldb + q];
                    else o[q] = row[q];
                }
                int z = 0;
                asm volatile("" : "+v"(z));
#pragma unroll
                for (int qc = 0; qc < AW; qc += QC) {
                    T nw[QC];
#pragma unroll
                    for (int j = 0; j < QC; ++j) nw[j] = T(0);
#pragma unroll
                    for (int q = 0; q < AW; ++q)
#pragma unroll
                        for (int j = 0; j < QC; ++j) nw[j] = fma(o[q], lds_m2[z + q * W + qc + j], nw[j]);
#pragma unroll
                    for (int j = 0; j < QC; ++j) row[qc + j] = nw[j];
                }
                if constexpr (PF) {
#pragma unroll
                    for (int q = 0; q < AW; ++q) o[q] = on[q];
                }
            }
            // M2q <- M2p M2: lane k forms row k (its row of M2p loaded once)
            const T *pa = a.M2p + (int64_t)item * W * W;
            T *pm = a.M2q + (int64_t)item * W * W;
            for (int k = lane; k < AW; k += kWave) {
                T r[AW];
#pragma unroll
                for (int q = 0; q < AW; ++q) r[q] = pa[k * W + q];
#pragma unroll
                for (int qc = 0; qc < AW; qc += QC) {
                    T acc[QC];
#pragma unroll
                    for (int j = 0; j < QC; ++j) acc[j] = T(0);
#pragma unroll
                    for (int q = 0; q < AW; ++q)
#pragma unroll
                        for (int j = 0; j < QC; ++j) acc[j] = fma(r[q], lds_m2[q * W + qc + j], acc[j]);
#pragma unroll
                    for (int j = 0; j < QC; ++j) pm[k * W + qc + j] = acc[j];
                }
            }
        }
    }
}

template <typename T>
struct ZupdArgsT {
    int r0;                    // rows r0 .. lo-1 are updated (r0 and lo even, lo - r0 >= 2)
    int lo;
    int c0;                    // first column of H in the block (lo - m)
    int K;                     // rows of M_blk multiplying H (n_b + m bottom, k n_b otherwise)
    int m;
    int nr;                    // right-hand-side columns carried after z (dense right-hand side: m), else 0
    int n;                     // order of H: columns past n-1 are never read
    int ncols;                 // columns of Z (W per work item, a multiple of 128)
    int count;                 // work items
    int has_zin;               // 0 for the bottom tile (no carried columns in Z yet)
    const T *H;                // ld ldh, 16-byte aligned columns
    int64_t ldh;
    const T *Bm;               // row-major, row stride ldb; rows K .. K rounded up to 16 are zero
    int64_t ldb;
    const T *M2;
    T *Z;
    int64_t ldz;
    const double *shifts;
    const int32_t *list;
    const int *dcount;         // if set, the number of work items is read here (count is an upper bound)
};
using ZupdArgs = ZupdArgsT<double>;

// What the direct-to-LDS loads assume: 16-byte aligned groups of rows of H
// and of columns of Bm (two doubles or four floats), at least one group of
// rows, K a whole number of chunks unless the padding rows of Bm are zero
// (the bottom tile).
template <typename T>
inline bool zupd_args_ok(int m, const ZupdArgsT<T> &a)
{
    constexpr int G = 16 / (int)sizeof(T);
    return !((a.r0 | a.lo) % G || a.lo - a.r0 < G || a.ldh % G || a.ldb % G || a.ncols % 128 != 0 ||
             a.ncols % zupd_bn(blk_cols(m, a.nr != 0)) != 0 || a.c0 < 0 ||
             (a.has_zin && a.K % 16 != 0 && a.nr == 0) || a.K <= 0 || a.n < a.lo ||
             ((uintptr_t)a.H | (uintptr_t)a.Bm) & 15 || (a.nr != 0 && a.nr != m));
}

typedef double zupd_dbl4 __attribute__((ext_vector_type(4)));

// LDS of zupd_kernel (dynamic): two stages of a 16 x 128 chunk of H^T rows
// and of Bm rows.
constexpr int kZupdLds = 2 * 2 * 16 * 128 * (int)sizeof(double);

// Z(0:lo, :) <- H(0:lo, c0 : c0+K) Bm(0:K, :) + (per shift) Z M2, minus
// sigma M1 on the rows whose diagonal is in the block.  128 x BN tiles
// (BN = zupd_bn(W): whole shifts per tile), 4 waves of 64 x BN/2 (4 x BN/32
// blocks of v_mfma_f64_16x16x4f64; lane l holds
// A(l%16, l/16), B(l/16, l%16); result register r of lane l is
// D(4r + l/16, l%16)).
//
// The carried part comes first: each wave loads its Z fragments in two
// batches (issued together, so one memory latency per batch) and
// multiplies them by M2 into the accumulators.  For W < 16 a 16-column
// block holds several shifts and M2 acts as a block-diagonal operand; the
// tile kernel keeps every shift's Z finite (a shift with a non-finite sigma
// gets a zero block transform), so the zeros never meet a NaN.  With W = 24
// a block may end inside one shift and start the next: its operand then
// covers both shifts' columns, again block-diagonal.  A
// workgroup reads only its own tile of Z (its shifts' columns), all before
// it writes, so the update is in place.
//
// The main product streams K in chunks of 16 through two LDS stages that
// the memory system fills directly (global_load_lds_dwordx4: each lane
// moves two consecutive doubles of one row of the chunk, so neither operand
// passes through registers).  Both operands sit in LDS k-major ([k][row]
// and [k][column]), which is how H (column-major) and Bm (row-major) lie in
// memory; the fragment reads of 16 consecutive rows or columns are free of
// bank conflicts.  Rows of the tile at or past lo read row lo-2 and columns
// past n-1 read column n-1: their products are never stored or meet zero
// rows of Bm.  An LDS row of Bm always takes 128 columns; with BN = 96 the
// lanes past the tile load its last two columns again.  Each chunk's loads
// are issued right after the previous chunk's fragments are in registers
// and waited for only after its 16 NT MFMAs.
template <int W>
__global__ __launch_bounds__(256, 2) void zupd_kernel(ZupdArgsT<double> a)
{
    constexpr int BM = 128, BN = zupd_bn(W), BK = 16;
    constexpr int NT = BN / 32;   // 16-column blocks per wave
    extern __shared__ double zupd_smem[];
    auto As = reinterpret_cast<double (*)[BK][BM]>(zupd_smem);
    auto Bs = reinterpret_cast<double (*)[BK][128]>(zupd_smem + 2 * BK * BM);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lo = a.lo, K = a.K;
    // Tile order.  Workgroup L of the 1-D grid runs on XCD L mod 8; each XCD
    // takes a contiguous chunk of the tile sequence, which walks groups of
    // 8 row tiles column by column.  The workgroups resident on one XCD then
    // share 8 row tiles of H and a few column tiles of Bm in its L2 (this
    // halves the kernel's HBM reads against a row-major launch order).
    int i0, j0;
    {
        const int nx = a.ncols / BN, ny = (lo - a.r0 + BM - 1) / BM, T = nx * ny;
        const int L = blockIdx.x, xcd = L & 7, li = L >> 3;
        const int per = T >> 3, rem = T & 7;
        const int g = xcd * per + min(xcd, rem) + li;
        constexpr int GR = 8;
        const int grp = g / (GR * nx), r = g - grp * GR * nx;
        const int rows = min(GR, ny - grp * GR);
        i0 = a.r0 + (grp * GR + r % rows) * BM;
        j0 = (r / rows) * BN;
    }
    const int count = a.dcount ? *a.dcount : a.count;
    if (j0 >= count * W) return;   // uniform: every column of the tile belongs to no listed item

    zupd_dbl4 acc[4][NT];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y) acc[x][y] = zupd_dbl4{0.0, 0.0, 0.0, 0.0};

    // ---- carried part: Z(rows, shift) * M2(shift) ------------------------------
    if (a.has_zin) {
        // Z columns feeding one 16-column block: the shifts the block touches
        // (W = 24: up to two, the second one's only where the block crosses
        // into it)
        constexpr int KZ = W > 16 ? (W % 16 ? 2 * W : W) : 16;
        constexpr int KP = KZ > 32 ? 16 : KZ;  // of them per pass (registers)
        constexpr int NS = KP / 4;            // MFMA k-steps per block and pass
#pragma unroll
        for (int kpass = 0; kpass < KZ / KP; ++kpass)
#pragma unroll
        for (int half = 0; half < (NT + 1) / 2; ++half) {
            double az[2][4][NS], bz[2][NS];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int nt = 2 * half + h;
                if (nt >= NT) break;
                const int cb = j0 + wc * (BN / 2) + nt * 16;   // first output column of the block
                const int zc = W <= 16 ? cb : (cb / W) * W;
                const int zend = W % 16 ? ((cb + 15) / W + 1) * W : zc + KZ;   // past the block's last shift
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int k = kpass * KP + 4 * s + lane / 16, q = lane % 16;
                    const bool kin = W % 16 == 0 || zc + k < zend;
                    if constexpr (W <= 16) {
                        const int sk = (cb + k) / W, sq = (cb + q) / W;
                        bz[h][s] = sk == sq ? a.M2[(int64_t)sk * W * W + ((cb + k) % W) * W + (cb + q) % W] : 0.0;
                    } else if constexpr (W % 16 != 0) {
                        const int zk = zc + k, sk = zk / W, sq = (cb + q) / W;
                        bz[h][s] = kin && sk == sq ? a.M2[(int64_t)sk * W * W + (zk % W) * W + (cb + q) % W] : 0.0;
                    } else {
                        bz[h][s] = a.M2[(int64_t)(cb / W) * W * W + k * W + cb % W + q];
                    }
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        const int i = i0 + wr * 64 + mt * 16 + lane % 16;
                        az[h][mt][s] = i < lo && kin ? a.Z[(int64_t)(zc + k) * a.ldz + i] : 0.0;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2 && 2 * half + h < NT; ++h)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        acc[mt][2 * half + h] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(az[h][mt][s], bz[h][s], acc[mt][2 * half + h], 0, 0, 0);
        }
    }

    // ---- main product: H(0:lo, c0 : c0+K) Bm -----------------------------------
    // wave w moves rows k = 4w .. 4w+3 of each chunk of both operands
    const int ia = min(i0 + 2 * lane, lo - 2);
    const double *pa = a.H + ia;
    const double *pb = a.Bm + j0 + min(2 * lane, BN - 2);
    auto issue = [&](int b, int k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * wave + e;
            const int col = min(a.c0 + k0 + k, a.n - 1);
            __builtin_amdgcn_global_load_lds((const void *)(pa + (int64_t)col * a.ldh),
                                             (__attribute__((address_space(3))) void *)&As[b][k][0], 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(pb + (int64_t)(k0 + k) * a.ldb),
                                             (__attribute__((address_space(3))) void *)&Bs[b][k][0], 16, 0, 0);
        }
    };
    const int nk = (K + BK - 1) / BK;
    if (nk > 0) issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0)
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const int b = it & 1;
        double af[4][4], bf[4][NT];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) af[s][mt] = As[b][4 * s + lane / 16][wr * 64 + mt * 16 + lane % 16];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bf[s][nt] = Bs[b][4 * s + lane / 16][wc * (BN / 2) + nt * 16 + lane % 16];
        }
        // the other stage was last read before the previous barrier
        if (it + 1 < nk) issue(b ^ 1, (it + 1) * BK);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[s][mt], bf[s][nt], acc[mt][nt], 0, 0, 0);
        // keep the wait for the next chunk behind this chunk's products
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0070);
        __syncthreads();
    }

    // ---- epilogue: sigma on the block's diagonal rows, store ----------------
    const int m = a.m;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr * 64 + mt * 16 + 4 * r + lane / 16;
                const int j = j0 + wc * (BN / 2) + nt * 16 + lane % 16;
                if (i >= lo) continue;
                double v = acc[mt][nt][r];
                if (i >= lo - m) {
                    const int w = j / W, q = j % W;
                    const int sid = w < count ? (a.list ? a.list[w] : w) : 0;
                    const double sr = a.shifts[2 * sid], si = a.shifts[2 * sid + 1];
                    // a non-finite sigma has a zero transform and keeps Z zero.
                    // Column pairs (re, im): (c, m + c) of the carried columns,
                    // (2m + c, 3m + c) of a dense right-hand side.
                    const int base = q < 2 * m ? 0 : 2 * m, qq = q - base, half = base ? a.nr : m;
                    if (w < count && qq < 2 * half && isfinite(sr) && isfinite(si)) {
                        const int c = qq < half ? qq : qq - half;
                        const int p = i - (lo - m);
                        const double ur = a.Bm[(int64_t)p * a.ldb + w * W + base + c];
                        const double ui = a.Bm[(int64_t)p * a.ldb + w * W + base + half + c];
                        v -= qq < half ? (sr * ur - si * ui) : (sr * ui + si * ur);
                    }
                }
                a.Z[(int64_t)j * a.ldz + i] = v;
            }
}


// FP32 form of zupd_kernel for the mixed-precision sweep: the same tiling,
// schedule and direct-to-LDS operand streaming, on H32 with
// v_mfma_f32_16x16x4f32 (twice the FP64 matrix rate).  Each direct-to-LDS
// load moves four consecutive floats per lane, so one instruction fills two
// k-rows of a chunk (lanes 0-31 the first, 32-63 the second).  The result
// layout of the FP32 instruction differs from the FP64 one: register r of
// lane l holds D(4 (l/16) + r, l%16).
typedef float zupd_flt4 __attribute__((ext_vector_type(4)));
constexpr int kZupd32Lds = 2 * 2 * 16 * 128 * (int)sizeof(float);

template <int W>
__global__ __launch_bounds__(256, 2) void zupd32_kernel(ZupdArgsT<float> a)
{
    constexpr int BM = 128, BN = zupd_bn(W), BK = 16;
    constexpr int NT = BN / 32;   // 16-column blocks per wave
    extern __shared__ float zupd32_smem[];
    auto As = reinterpret_cast<float (*)[BK][BM]>(zupd32_smem);
    auto Bs = reinterpret_cast<float (*)[BK][128]>(zupd32_smem + 2 * BK * BM);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lo = a.lo, K = a.K;
    int i0, j0;
    {
        const int nx = a.ncols / BN, ny = (lo - a.r0 + BM - 1) / BM, T = nx * ny;
        const int L = blockIdx.x, xcd = L & 7, li = L >> 3;
        const int per = T >> 3, rem = T & 7;
        const int g = xcd * per + min(xcd, rem) + li;
        constexpr int GR = 8;
        const int grp = g / (GR * nx), r = g - grp * GR * nx;
        const int rows = min(GR, ny - grp * GR);
        i0 = a.r0 + (grp * GR + r % rows) * BM;
        j0 = (r / rows) * BN;
    }
    const int count = a.dcount ? *a.dcount : a.count;
    if (j0 >= count * W) return;

    zupd_flt4 acc[4][NT];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y) acc[x][y] = zupd_flt4{0.f, 0.f, 0.f, 0.f};

    // ---- carried part: Z(rows, shift) * M2(shift) ------------------------------
    if (a.has_zin) {
        // Z columns feeding one 16-column block: the shifts the block touches
        // (W = 24: up to two, the second one's only where the block crosses
        // into it)
        constexpr int KZ = W > 16 ? (W % 16 ? 2 * W : W) : 16;
        constexpr int KP = KZ > 32 ? 16 : KZ;  // of them per pass (registers)
        constexpr int NS = KP / 4;            // MFMA k-steps per block and pass
#pragma unroll
        for (int kpass = 0; kpass < KZ / KP; ++kpass)
#pragma unroll
        for (int half = 0; half < (NT + 1) / 2; ++half) {
            float az[2][4][NS], bz[2][NS];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int nt = 2 * half + h;
                if (nt >= NT) break;
                const int cb = j0 + wc * (BN / 2) + nt * 16;
                const int zc = W <= 16 ? cb : (cb / W) * W;
                const int zend = W % 16 ? ((cb + 15) / W + 1) * W : zc + KZ;   // past the block's last shift
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int k = kpass * KP + 4 * s + lane / 16, q = lane % 16;
                    const bool kin = W % 16 == 0 || zc + k < zend;
                    if constexpr (W <= 16) {
                        const int sk = (cb + k) / W, sq = (cb + q) / W;
                        bz[h][s] = sk == sq ? a.M2[(int64_t)sk * W * W + ((cb + k) % W) * W + (cb + q) % W] : 0.f;
                    } else if constexpr (W % 16 != 0) {
                        const int zk = zc + k, sk = zk / W, sq = (cb + q) / W;
                        bz[h][s] = kin && sk == sq ? a.M2[(int64_t)sk * W * W + (zk % W) * W + (cb + q) % W] : 0.f;
                    } else {
                        bz[h][s] = a.M2[(int64_t)(cb / W) * W * W + k * W + cb % W + q];
                    }
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) {
                        const int i = i0 + wr * 64 + mt * 16 + lane % 16;
                        az[h][mt][s] = i < lo && kin ? a.Z[(int64_t)(zc + k) * a.ldz + i] : 0.f;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2 && 2 * half + h < NT; ++h)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        acc[mt][2 * half + h] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(az[h][mt][s], bz[h][s], acc[mt][2 * half + h], 0, 0, 0);
        }
    }

    // ---- main product: H(0:lo, c0 : c0+K) Bm -----------------------------------
    // wave w moves k-rows 4w .. 4w+3 of each chunk of both operands, two per
    // instruction (lane l: k-row 4w + 2e + l/32, elements 4 (l%32) .. + 3)
    const int hk = lane >> 5, p4 = 4 * (lane & 31);
    const int ia = min(i0 + p4, lo - 4);
    const float *pa = a.H + ia;
    const float *pb = a.Bm + j0 + min(p4, BN - 4);
    auto issue = [&](int b, int k0) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int k = 4 * wave + 2 * e + hk;
            const int col = min(a.c0 + k0 + k, a.n - 1);
            __builtin_amdgcn_global_load_lds((const void *)(pa + (int64_t)col * a.ldh),
                                             (__attribute__((address_space(3))) void *)&As[b][4 * wave + 2 * e][0], 16,
                                             0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(pb + (int64_t)(k0 + k) * a.ldb),
                                             (__attribute__((address_space(3))) void *)&Bs[b][4 * wave + 2 * e][0], 16,
                                             0, 0);
        }
    };
    const int nk = (K + BK - 1) / BK;
    if (nk > 0) issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0)
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const int b = it & 1;
        float af[4][4], bf[4][NT];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) af[s][mt] = As[b][4 * s + lane / 16][wr * 64 + mt * 16 + lane % 16];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bf[s][nt] = Bs[b][4 * s + lane / 16][wc * (BN / 2) + nt * 16 + lane % 16];
        }
        if (it + 1 < nk) issue(b ^ 1, (it + 1) * BK);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[s][mt], bf[s][nt], acc[mt][nt], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0070);
        __syncthreads();
    }

    // ---- epilogue: sigma on the block's diagonal rows, store ----------------
    const int m = a.m;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr * 64 + mt * 16 + 4 * (lane / 16) + r;
                const int j = j0 + wc * (BN / 2) + nt * 16 + lane % 16;
                if (i >= lo) continue;
                float v = acc[mt][nt][r];
                if (i >= lo - m) {
                    const int w = j / W, q = j % W;
                    const int sid = w < count ? (a.list ? a.list[w] : w) : 0;
                    const float sr = (float)a.shifts[2 * sid], si = (float)a.shifts[2 * sid + 1];
                    const int base = q < 2 * m ? 0 : 2 * m, qq = q - base, half = base ? a.nr : m;
                    if (w < count && qq < 2 * half && isfinite(sr) && isfinite(si)) {
                        const int c = qq < half ? qq : qq - half;
                        const int p = i - (lo - m);
                        const float ur = a.Bm[(int64_t)p * a.ldb + w * W + base + c];
                        const float ui = a.Bm[(int64_t)p * a.ldb + w * W + base + half + c];
                        v -= qq < half ? (sr * ur - si * ui) : (sr * ui + si * ur);
                    }
                }
                a.Z[(int64_t)j * a.ldz + i] = v;
            }
}

}  // namespace shs
