// Per-shift RQ sweep of H - sigma I with an (m+1)-column sliding window.
//
// Section 3.1 factors H - sigma I = R_sigma Q_sigma from the bottom row to
// the top row, keeping only a narrow window of columns, because only the
// leading m x m block of R_sigma is needed (Section 3, introduction).  Here
// the window advances one column per step (block size 1) and each step uses
// one Householder reflector of size m+1 instead of the paper's Givens
// schedule:
//
//   step k = n-1 .. 0 (0-based), window = columns k-m .. k (columns < 0 are
//   zero):
//     1. row k of the window, w = W(k, :), defines a Hermitian reflector
//        P_k = I - tau v v^*, v_m = 1, with w P_k = beta_k e_m^T;
//        beta_k = R_sigma(k, k);
//     2. every row i < k: r <- r P_k, i.e. r -= tau (r v) v^*;
//     3. column k leaves the window (its entries for rows i < k are
//        R_sigma(i, k)); the fresh column k-1-m of H enters, with -sigma on
//        the diagonal (the sigma-diagonal kernels of Algorithm 8 are folded
//        into this load).
//
//   After step k = 0, (H - sigma I) P_{n-1} ... P_0 = R_sigma, so
//   X = P_{n-1} ... P_0 [Y; 0] with Y = R_sigma(0:m,0:m)^{-1} R(0:m,:).
//   The back-substitution for Y is fused into the last m steps: after step
//   k < m, y_k = e_k / beta_k and e_i -= R_sigma(i, k) y_k for i < k, where
//   e starts as R(0:m, 0:m) (Section 3.1, last paragraph: one step of the
//   reduction followed by one step of the back substitution).
//
//   DENSE = true solves (H - sigma I) D = E for a dense n x m right-hand side
//   E (the correction solve of iterative refinement): every row carries
//   e_i = E(i, :), and every step k does y_k = e_k / beta_k (stored beside
//   the reflector) and e_i -= R_sigma(i, k) y_k for the rows above it: the
//   column-oriented back substitution with the full triangle of R_sigma,
//   done on the fly as the dense-right-hand-side solver of Section 3.3 does
//   with its triangular factor.
//
// GPU mapping: one wavefront per shift.  Rows are processed in tiles of
// T = 64 R rows from the bottom tile to the top one; lane l of the wave owns
// rows lo + 64 r + l (r < R) and keeps their window rows in registers.  A
// tile first replays the reflectors already produced by the tiles below it
// (its rows are above all of their pivots, so every replay is a pure
// per-lane update with the reflector broadcast to all lanes from LDS), then
// produces its own T reflectors, reading each pivot row out of its owner
// lane.  The reflectors go to a per-shift store in HBM that later tiles and
// the Q* pass read back.  The window rotates through the registers: logical
// window position j of step k sits in register slot (j + k) mod (m+1), so
// nothing moves when the window slides; every step body is instantiated for
// its phase k mod (m+1), and all register indices are compile-time
// constants.
#pragma once

#include <utility>

#include <limits>

#include "common.hpp"

namespace shs {

// Calls f(std::integral_constant<int, s>) for s = 0 .. N-1.
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    [&]<int... S>(std::integer_sequence<int, S...>) {
        (f(std::integral_constant<int, S>{}), ...);
    }(std::make_integer_sequence<int, N>{});
}

// Reflector-store layout of one shift: the slots of row tile t start at
// t * tile_stride (a multiple of 256 bytes), slot k of the tile at
// (k - t T) * slot_elems.  Keeping tiles on separate cache lines means a
// tile's slots are never in a line that was cached before they were written.
template <typename T>
__host__ __device__ inline int64_t refl_tile_stride(int rows_per_tile, int slot)
{
    const int64_t bytes = (int64_t)rows_per_tile * slot * (int64_t)sizeof(T);
    return ((bytes + 255) / 256) * 256 / (int64_t)sizeof(T);
}

template <typename T>
struct SweepArgs {
    int n;
    int count;                 // number of work items (= launched workgroups)
    const T *H;                // column-major n x n, leading dimension ldh
    int64_t ldh;
    const double *shifts;      // interleaved complex, indexed by shift id
    const int32_t *list;       // work item -> shift id, nullptr = identity
    const double *Rtop;        // structured: m x m upper triangle of R (ld m)
    const T *E;                // dense: per shift id, n x m complex (ld n)
    int64_t e_stride;          // elements between shifts in E
    T *refl;                   // per shift id: ceil(n / T) tiles of tile_stride
    int64_t refl_stride;
    T *Y;                      // structured: m x m complex (ld m); dense: n x m (ld n)
    int64_t y_stride;
    int32_t *status;           // per shift id
    const int *dcount;         // if set, the number of work items is read here (count is then an upper bound)
};

// Compile-time shape of one kernel instance.
template <typename T, int M, bool DENSE, int RB = 0>
struct SweepShape {
    // RB > 0 overrides the rows per lane (the blocked tile kernels)
    static constexpr int R = RB > 0 ? RB : rows_per_lane<T, M, DENSE>();
    static constexpr int TT = kWave * R;
    static constexpr int S = slot_elems(M, DENSE);
    static constexpr int EM = DENSE ? M : 1;
    static constexpr int NP = M + 1;
    // The replay streams reflectors through LDS in chunks of KC steps, a
    // whole number of phase groups, starting at a multiple of KC.
    static constexpr int KC = ((16 + NP - 1) / NP) * NP;
    static constexpr int CH = KC * S;                    // elements per chunk
    static constexpr int PL = (CH + kWave - 1) / kWave;  // elements per lane
};

template <typename T>
__device__ __forceinline__ const T *refl_slot(const T *rf, int k, int tt, int64_t tstride, int S)
{
    const int t = k / tt;
    return rf + (int64_t)t * tstride + (int64_t)(k - t * tt) * S;
}

// Fresh column `col` of H for this lane's rows.  Rows past n (the ragged
// bottom tile) read row n-1 instead: they are never pivots and never feed
// another row, so their values do not matter, and the loads stay free of
// per-lane branches.  A negative col reads column 0, and the consumer
// (apply_step) takes zeros instead; the loads are so issued on every step,
// and with no branch around them the waits for them count exactly the
// memory operations issued since.
template <typename T, int M, int R>
__device__ __forceinline__ void load_fresh(const T *H, int64_t ldh, int n, int lo, int lane, int col,
                                           T (&fr)[R])
{
    if constexpr (M == 1) {
        // one-column windows in eight row slots: here the unconditional
        // loads let the compiler keep too many of them live, so a negative
        // col skips them (the waits are then counted less exactly)
        if (col < 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) fr[r] = T(0);
            return;
        }
    }
    const T *cp = H + (int64_t)(col < 0 ? 0 : col) * ldh;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lo + r * kWave + lane;
        fr[r] = cp[i < n ? i : n - 1];
    }
}

// Reflector from a pivot row w (logical order, w[m] = column k).
// x = conj(w); alpha = x_m; P x = beta' e_m with P Hermitian, so
// w P = conj(beta') e_m^T.  With u = x - beta' e_m scaled to u_m = 1:
// v_j = conj(w_j) / u_m, tau = 2 |u_m|^2 / ||u||^2.  A row that is already
// [0 ... 0 w_m] gives tau = 0 (P = I) and beta = w_m.
//
// With a = |alpha|, phase ph = alpha / a (1 when a = 0), nu = ||x|| and
// u_m = ph (a + nu): ||u||^2 = 2 nu (a + nu), so tau = (a + nu) / nu, and
// 1 / u_m = conj(ph) / (a + nu) = conj(alpha) / (a (a + nu)): two
// reciprocal square roots and two reciprocals per reflector.
template <typename T, int M>
__device__ __forceinline__ void make_refl(const T (&pr)[M + 1], const T (&pi)[M + 1], T (&vr)[M], T (&vi)[M],
                                          T &tau, T &br, T &bi)
{
    T sig2 = T(0);
#pragma unroll
    for (int j = 0; j < M; ++j) sig2 = fma(pr[j], pr[j], fma(pi[j], pi[j], sig2));
    const T ar = pr[M], ai = -pi[M];
    // no branch for the already-reduced row (sig2 = 0): there x_j = 0, so v
    // comes out zero as long as the scale below is finite, and tau and beta
    // are selected.  Square roots and reciprocals come from the hardware
    // estimates with Newton steps (rsq_nr, rcp_nr); an alpha below the
    // smallest normal counts as zero (phase 1), which moves u_m by at most
    // that much.
    const bool z = sig2 == T(0);
    const T a2 = fma(ar, ar, ai * ai), n2 = a2 + sig2;
    const bool ph = a2 >= std::numeric_limits<T>::min();
    const T ia = ph ? rsq_nr<T>(ph ? a2 : T(1)) : T(0);    // 1 / |alpha|
    const T aa = a2 * ia;                                  // |alpha|
    const bool nz = n2 >= std::numeric_limits<T>::min();
    const T nu = nz ? n2 * rsq_nr<T>(nz ? n2 : T(1)) : T(0);   // ||x||
    const T um = aa + nu;                                  // |u_m|
    const T ru = um > T(0) ? rcp_nr<T>(um > T(0) ? um : T(1)) : T(0);
    // cr - i ci = conj(u_m) / |u_m|^2 = conj(ph) / um (zero for a zero row)
    const T cr = ph ? ar * ia * ru : ru, ci = ph ? ai * ia * ru : T(0);
    tau = z ? T(0) : um * rcp_nr<T>(nz ? nu : T(1));
    // beta = -ph nu (as conj(beta') e_m^T = w P), ph = (cr + i ci) um;
    // w_m itself when P = I
    const T s = nu * um;
    br = z ? pr[M] : -cr * s;
    bi = z ? pi[M] : ci * s;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        // conj(w_j) * conj(u_m) / |u_m|^2
        const T xr = pr[j], xi = -pi[j];
        vr[j] = fma(xr, cr, xi * ci);
        vi[j] = fma(xi, cr, -(xr * ci));
    }
}

// Apply P_k to row slots [0, RA) at phase Q = k mod (m+1), then slide: the
// freed register takes the fresh column (fcol, with -sigma on the diagonal).
// DENSE rows also do e -= R_sigma(i, k) y_k; DROP returns R_sigma(i, k) of
// slot 0 in (d0r, d0i).
template <typename T, int M, int R, int EM, int Q, int RA, bool DENSE, bool DROP>
__device__ __forceinline__ void apply_step(T (&wr)[R][M + 1], T (&wi)[R][M + 1], T (&er)[R][EM],
                                           T (&ei)[R][EM], const T (&vr)[M], const T (&vi)[M], T tau,
                                           const T (&yr)[EM], const T (&yi)[EM], const T (&fr)[R],
                                           int fcol, int lo, int lane, T sgr, T sgi, T &d0r, T &d0i)
{
    constexpr int NP = M + 1;
    constexpr int pm = (M + Q) % NP;
#pragma unroll
    for (int r = 0; r < RA; ++r) {
        T dr = wr[r][pm], di = wi[r][pm];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int p = (j + Q) % NP;
            dr = fma(wr[r][p], vr[j], dr);
            dr = fma(-wi[r][p], vi[j], dr);
            di = fma(wr[r][p], vi[j], di);
            di = fma(wi[r][p], vr[j], di);
        }
        const T tr = tau * dr, ti = tau * di;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int p = (j + Q) % NP;
            // w_j -= t conj(v_j)
            wr[r][p] = fma(-tr, vr[j], fma(-ti, vi[j], wr[r][p]));
            wi[r][p] = fma(-ti, vr[j], fma(tr, vi[j], wi[r][p]));
        }
        if constexpr (DENSE || DROP) {
            // the column that leaves: R_sigma(i, k) = w_m - t
            const T xr = wr[r][pm] - tr, xi = wi[r][pm] - ti;
            if constexpr (DENSE) {
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    er[r][c] = fma(-xr, yr[c], fma(xi, yi[c], er[r][c]));
                    ei[r][c] = fma(-xr, yi[c], fma(-xi, yr[c], ei[r][c]));
                }
            }
            if (r == 0) { d0r = xr; d0i = xi; }
        }
        const T f = fcol >= 0 ? fr[r] : T(0);   // columns left of 0 are zero
        if (fcol >= lo && fcol < lo + R * kWave) {   // uniform: a diagonal entry enters
            const bool dg = (lo + r * kWave + lane) == fcol;
            wr[r][pm] = dg ? f - sgr : f;
            wi[r][pm] = dg ? -sgi : T(0);
        } else {
            wr[r][pm] = f;
            wi[r][pm] = T(0);
        }
    }
}

// Pivot row of step k (local index q in the tile), read out of its owner
// lane: every slot's candidate is read with readlane (uniform lane index)
// and the slot is then chosen with uniform selects, so every register index
// stays static.  RS = R reads only slot 0 (the pivot is known to be there).
template <typename T, int M, int R, int EM, int Q, bool DENSE, int RS = R>
__device__ __forceinline__ void pivot_row(const T (&wr)[R][M + 1], const T (&wi)[R][M + 1],
                                          const T (&er)[R][EM], const T (&ei)[R][EM], int q,
                                          T (&pr)[M + 1], T (&pi)[M + 1], T (&pe_r)[EM], T (&pe_i)[EM])
{
    constexpr int NP = M + 1;
    const int rp = q >> 6, lp = q & 63;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        T xr = readlane(wr[0][(j + Q) % NP], lp), xi = readlane(wi[0][(j + Q) % NP], lp);
#pragma unroll
        for (int r = 1; r < RS; ++r) {
            const T yr = readlane(wr[r][(j + Q) % NP], lp), yi = readlane(wi[r][(j + Q) % NP], lp);
            xr = rp == r ? yr : xr;
            xi = rp == r ? yi : xi;
        }
        pr[j] = xr;
        pi[j] = xi;
    }
    if constexpr (DENSE) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T xr = readlane(er[0][c], lp), xi = readlane(ei[0][c], lp);
#pragma unroll
            for (int r = 1; r < RS; ++r) {
                const T yr = readlane(er[r][c], lp), yi = readlane(ei[r][c], lp);
                xr = rp == r ? yr : xr;
                xi = rp == r ? yi : xi;
            }
            pe_r[c] = xr;
            pe_i[c] = xi;
        }
    }
}

// Pivot row when its slot RP is known at compile time: NP readlanes of that
// slot only.
template <typename T, int M, int R, int EM, int Q, bool DENSE, int RP>
__device__ __forceinline__ void pivot_row_slot(const T (&wr)[R][M + 1], const T (&wi)[R][M + 1],
                                               const T (&er)[R][EM], const T (&ei)[R][EM], int lp,
                                               T (&pr)[M + 1], T (&pi)[M + 1], T (&pe_r)[EM], T (&pe_i)[EM])
{
    constexpr int NP = M + 1;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        pr[j] = readlane(wr[RP][(j + Q) % NP], lp);
        pi[j] = readlane(wi[RP][(j + Q) % NP], lp);
    }
    if constexpr (DENSE) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            pe_r[c] = readlane(er[RP][c], lp);
            pe_i[c] = readlane(ei[RP][c], lp);
        }
    }
}

// One tile step k (phase Q = k mod (m+1)); RP >= 0: the pivot is known to
// be in slot RP, and only slots 0 .. RP are updated.
template <typename T, int M, bool DENSE, int Q, int RP, int RB = 0>
__device__ __forceinline__ void tri_step(int k, int k_lo, int n, int lo, int lane, const T *H, int64_t ldh, T sgr,
                                         T sgi, T *rf, int64_t tstride, T *Y, T *lds_rs,
                                         T (&wr)[SweepShape<T, M, DENSE, RB>::R][M + 1],
                                         T (&wi)[SweepShape<T, M, DENSE, RB>::R][M + 1],
                                         T (&er)[SweepShape<T, M, DENSE, RB>::R][SweepShape<T, M, DENSE, RB>::EM],
                                         T (&ei)[SweepShape<T, M, DENSE, RB>::R][SweepShape<T, M, DENSE, RB>::EM],
                                         T (&nh)[SweepShape<T, M, DENSE, RB>::R], bool &singular, bool &nonfinite)
{
    using Sh = SweepShape<T, M, DENSE, RB>;
    constexpr int R = Sh::R, TT = Sh::TT, S = Sh::S, EM = Sh::EM, NP = Sh::NP;
    T ch[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ch[r] = nh[r];
    const int kn = k - 1 >= k_lo ? k - 1 : k_lo;
    load_fresh<T, M, R>(H, ldh, n, lo, lane, kn - 1 - M, nh);
    T pr[NP], pi[NP], per[EM], pei[EM];
    if constexpr (RP < 0)
        pivot_row<T, M, R, EM, Q, DENSE>(wr, wi, er, ei, k - lo, pr, pi, per, pei);
    else
        pivot_row_slot<T, M, R, EM, Q, DENSE, (RP < 0 ? 0 : RP)>(wr, wi, er, ei, (k - lo) & 63, pr,
                                                              pi, per, pei);
    T vr[M], vi[M], tau, br, bi, yr[EM], yi[EM];
    make_refl<T, M>(pr, pi, vr, vi, tau, br, bi);
    if (br == T(0) && bi == T(0)) singular = true;
    if constexpr (DENSE) {
        const T den = T(1) / fma(br, br, bi * bi);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            yr[c] = (per[c] * br + pei[c] * bi) * den;
            yi[c] = (pei[c] * br - per[c] * bi) * den;
            if (!isfinite(yr[c]) || !isfinite(yi[c])) nonfinite = true;
        }
    } else {
        yr[0] = T(0);
        yi[0] = T(0);
    }
    {
        // every lane stores the same (uniform) values: no branch around the
        // stores, so the waits for the fresh-column loads stay exact
        T *p = const_cast<T *>(refl_slot<T>(rf, k, TT, tstride, S));
        p[0] = tau;
        p[1] = T(0);
#pragma unroll
        for (int j = 0; j < M; ++j) { p[2 + 2 * j] = vr[j]; p[3 + 2 * j] = vi[j]; }
    }
    if (lane == 0) {
        T *p = const_cast<T *>(refl_slot<T>(rf, k, TT, tstride, S));
        if constexpr (DENSE) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                p[2 + 2 * M + 2 * c] = yr[c];
                p[3 + 2 * M + 2 * c] = yi[c];
                Y[2 * ((int64_t)c * n + k)] = yr[c];
                Y[2 * ((int64_t)c * n + k) + 1] = yi[c];
            }
        }
    }
    T dr0 = T(0), di0 = T(0);
    apply_step<T, M, R, EM, Q, (RP < 0 ? R : RP + 1), DENSE, !DENSE>(
        wr, wi, er, ei, vr, vi, tau, yr, yi, ch, k - 1 - M, lo, lane, sgr, sgi, dr0, di0);
    if constexpr (!DENSE) {
        // leading block: R_sigma(i, k) for rows i < k (lanes of
        // slot 0 in the top tile) and beta_k on the diagonal
        if (k < M) {
            if (lane < k) {
                lds_rs[2 * (k * M + lane)] = dr0;
                lds_rs[2 * (k * M + lane) + 1] = di0;
            }
            if (lane == 0) {
                lds_rs[2 * (k * M + k)] = br;
                lds_rs[2 * (k * M + k) + 1] = bi;
            }
        }
    }
}

// The tile's own steps k = hi-1 .. lo: each pivot row is read out of its
// owner lane, its reflector is formed, stored (lane 0) and applied to the
// tile's rows above it.  The top tile records the leading block of R_sigma
// (rows and columns < m) in lds_rs for the back substitution.
//
// SLOTS = true walks the steps slot by slot (pivots in slot R-1 first): the
// pivot slot is then a compile-time constant, so the pivot row costs m+1
// readlanes of one slot instead of all of them, and each step updates only
// slots 0 .. RP, the ones that still hold rows above the pivot (rows in
// higher slots are finished).  It unrolls the step body R times over; the
// per-shift sweep keeps the plain form, because beside its stream phase the
// R copies spill in FP32 (R = 8 there).
template <typename T, int M, bool DENSE, bool SLOTS = false, int RB = 0>
__device__ __forceinline__ void tri_phase(int n, int lo, int hi, int lane, const T *H, int64_t ldh, T sgr, T sgi,
                                          T *rf, int64_t tstride, T *Y, T *lds_rs,
                                          T (&wr)[SweepShape<T, M, DENSE, RB>::R][M + 1],
                                          T (&wi)[SweepShape<T, M, DENSE, RB>::R][M + 1],
                                          T (&er)[SweepShape<T, M, DENSE, RB>::R][SweepShape<T, M, DENSE, RB>::EM],
                                          T (&ei)[SweepShape<T, M, DENSE, RB>::R][SweepShape<T, M, DENSE, RB>::EM],
                                          bool &singular, bool &nonfinite)
{
    using Sh = SweepShape<T, M, DENSE, RB>;
    constexpr int R = Sh::R, TT = Sh::TT, S = Sh::S, EM = Sh::EM, NP = Sh::NP;
    const int k_end = lo;
    if (hi - 1 >= k_end) {
        const int k_hi = hi - 1, k_lo = k_end;
        T nh[R];
        load_fresh<T, M, R>(H, ldh, n, lo, lane, k_hi - 1 - M, nh);
        if constexpr (!SLOTS) {
            const int kg0 = k_hi + (M - k_hi % NP);   // group top: k = M (mod m+1)
            for (int kg = kg0; kg >= k_lo; kg -= NP) {
                static_for<NP>([&](auto sc) {
                    constexpr int st = decltype(sc)::value;
                    const int k = kg - st;
                    if (k <= k_hi && k >= k_lo)
                        tri_step<T, M, DENSE, M - st, -1, RB>(k, k_lo, n, lo, lane, H, ldh, sgr, sgi, rf, tstride, Y,
                                                          lds_rs, wr, wi, er, ei, nh, singular, nonfinite);
                });
            }
        } else {
            static_for<R>([&](auto rc) {
                constexpr int RP = R - 1 - decltype(rc)::value;
                const int s_lo = max(k_lo, lo + RP * kWave), s_hi = min(k_hi, lo + RP * kWave + kWave - 1);
                if (s_hi >= s_lo) {
                    const int kg0 = s_hi + (M - s_hi % NP);
                    for (int kg = kg0; kg >= s_lo; kg -= NP) {
                        static_for<NP>([&](auto sc) {
                            constexpr int st = decltype(sc)::value;
                            const int k = kg - st;
                            if (k <= s_hi && k >= s_lo)
                                tri_step<T, M, DENSE, M - st, RP, RB>(k, k_lo, n, lo, lane, H, ldh, sgr, sgi, rf, tstride,
                                                                  Y, lds_rs, wr, wi, er, ei, nh, singular, nonfinite);
                        });
                    }
                }
            });
        }
    }

}

// After the last step: the back substitution Y = R_sigma(0:m,0:m)^{-1} R(0:m,0:m)
// (structured right-hand side) from the leading block left in lds_rs, the
// shift's status, and NaN outputs for a singular shift.
template <typename T, int M, bool DENSE>
__device__ __forceinline__ void finish_shift(int n, int lane, const double *Rtop, T *Y, const T *lds_rs,
                                             int32_t *status, bool singular, bool nonfinite)
{
    // ---- back substitution Y = R_sigma(0:m,0:m)^{-1} R(0:m,0:m) -----------
    // The last m steps left the leading block of R_sigma and its diagonal in
    // LDS; lane c < m solves for column c of Y (structured right-hand side).
    if constexpr (!DENSE) {
        if (lane < M) {
            const int c = lane;
            T e_r[M], e_i[M];
#pragma unroll
            for (int i = 0; i < M; ++i) { e_r[i] = (T)Rtop[c * M + i]; e_i[i] = T(0); }
#pragma unroll
            for (int k = M - 1; k >= 0; --k) {
                const T br = lds_rs[2 * (k * M + k)], bi = lds_rs[2 * (k * M + k) + 1];
                const T den = T(1) / fma(br, br, bi * bi);
                const T yr = (e_r[k] * br + e_i[k] * bi) * den;
                const T yi = (e_i[k] * br - e_r[k] * bi) * den;
                if (!isfinite(yr) || !isfinite(yi)) nonfinite = true;
                Y[2 * (c * M + k)] = yr;
                Y[2 * (c * M + k) + 1] = yi;
#pragma unroll
                for (int i = 0; i < k; ++i) {
                    const T rr = lds_rs[2 * (k * M + i)], ri = lds_rs[2 * (k * M + i) + 1];
                    e_r[i] = fma(-rr, yr, fma(ri, yi, e_r[i]));
                    e_i[i] = fma(-rr, yi, fma(-ri, yr, e_i[i]));
                }
            }
        }
        // any lane's non-finite result marks the shift
        nonfinite = __any(nonfinite);
    }

    if (lane == 0) *status = singular ? 1 : (nonfinite ? 2 : 0);
    if (singular) {
        // no solution exists: NaN outputs for this shift only
        const T qnan = (T)__builtin_nan("");
        const int64_t cnt = DENSE ? (int64_t)n * M : (int64_t)M * M;
        for (int64_t idx = lane; idx < cnt; idx += kWave) {
            Y[2 * idx] = qnan;
            Y[2 * idx + 1] = qnan;
        }
    }
}

// One shift's sweep: everything one wavefront needs.
template <typename T>
struct SweepItem {
    int n;
    const T *H;            // column-major n x n
    int64_t ldh;
    T sgr, sgi;            // the shift
    T *rf;                 // this shift's reflector store
    T *Y;                  // structured: m x m (ld m); dense: n x m (ld n)
    const T *E;            // dense right-hand side n x m (ld n)
    const double *Rtop;    // structured: m x m leading block of R (ld m)
    int32_t *status;       // this shift's status
};

// LDS a sweep body needs (elements of T): reflector chunk + R_sigma block.
template <typename T, int M, bool DENSE>
__host__ __device__ constexpr int sweep_lds_elems()
{
    return SweepShape<T, M, DENSE>::CH + (DENSE ? 2 : 2 * M * M);
}

template <typename T, int M, bool DENSE>
__device__ __forceinline__ void sweep_body(const SweepItem<T> &it, T *lds_refl, T *lds_rs)
{
    using Sh = SweepShape<T, M, DENSE>;
    constexpr int R = Sh::R, TT = Sh::TT, S = Sh::S, EM = Sh::EM, NP = Sh::NP;
    constexpr int KC = Sh::KC, CH = Sh::CH, PL = Sh::PL;
    const int lane = threadIdx.x;
    const int n = it.n;
    const T *H = it.H;
    const int64_t ldh = it.ldh;
    const T sgr = it.sgr, sgi = it.sgi;
    T *rf = it.rf;
    T *Y = it.Y;
    const int64_t tstride = refl_tile_stride<T>(TT, S);

    T wr[R][NP], wi[R][NP];
    T er[R][EM], ei[R][EM];
    T dummy_r = T(0), dummy_i = T(0);
    bool singular = false, nonfinite = false;

    const int ntiles = (n + TT - 1) / TT;
    for (int t = ntiles - 1; t >= 0; --t) {
        const int lo = t * TT;
        const int hi = min(n, lo + TT);

        // ---- initial window of the tile's rows: columns n-1-m .. n-1 -------
        // Register slot p holds logical position (p - (n-1)) mod (m+1); the
        // column is computed per slot so that register indices stay static.
        {
            const int q0 = (n - 1) % NP;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int j = (p - q0 + NP) % NP;
                const int col = n - 1 - M + j;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = lo + r * kWave + lane;
                    T v = (col >= 0 && i < n) ? H[(int64_t)col * ldh + i] : T(0);
                    const bool dg = (i == col);
                    wr[r][p] = dg ? v - sgr : v;
                    wi[r][p] = dg ? -sgi : T(0);
                }
            }
            if constexpr (DENSE) {
                const T *E = it.E;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = lo + r * kWave + lane;
#pragma unroll
                    for (int c = 0; c < M; ++c) {
                        er[r][c] = i < n ? E[2 * ((int64_t)c * n + i)] : T(0);
                        ei[r][c] = i < n ? E[2 * ((int64_t)c * n + i) + 1] : T(0);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) { er[r][0] = T(0); ei[r][0] = T(0); }
            }
        }

        // ---- replay the reflectors of the tiles below: steps n-1 .. hi ------
        // Chunks of KC steps start at multiples of KC (a multiple of m+1), so
        // step kb + KC - 1 - st has phase (KC - 1 - st) mod (m+1).
        if (hi <= n - 1) {
            const int k_hi = n - 1, k_lo = hi;
            int kb = (k_hi / KC) * KC;
            T pre[PL];
            // slots outside [k_lo, k_hi] are loaded from a clamped (valid)
            // address and never read back
            auto fetch = [&](int base) {
#pragma unroll
                for (int e = 0; e < PL; ++e) {
                    const int idx0 = e * kWave + lane;
                    const int idx = idx0 < CH ? idx0 : CH - 1;
                    const int ks = idx / S, el = idx - ks * S;
                    int k = base + ks;
                    k = k < k_lo ? k_lo : (k > k_hi ? k_hi : k);
                    pre[e] = refl_slot(rf, k, TT, tstride, S)[el];
                }
            };
            fetch(kb);
            T nh[R];
            load_fresh<T, M, R>(H, ldh, n, lo, lane, k_hi - 1 - M, nh);
            for (; kb + KC - 1 >= k_lo; kb -= KC) {
                // one wave per workgroup: its LDS operations complete in
                // order, so the chunk can overwrite the previous one in place
#pragma unroll
                for (int e = 0; e < PL; ++e) {
                    const int idx = e * kWave + lane;
                    if (idx < CH) lds_refl[idx] = pre[e];
                }
                if (kb - 1 >= k_lo) fetch(kb - KC);
                static_for<KC>([&](auto sc) {
                    constexpr int st = decltype(sc)::value;
                    constexpr int Q = (KC - 1 - st) % NP;
                    const int k = kb + KC - 1 - st;
                    if (k <= k_hi && k >= k_lo) {
                        T ch[R];
#pragma unroll
                        for (int r = 0; r < R; ++r) ch[r] = nh[r];
                        const int kn = k - 1 >= k_lo ? k - 1 : k_lo;
                        load_fresh<T, M, R>(H, ldh, n, lo, lane, kn - 1 - M, nh);
                        const T *p = lds_refl + (KC - 1 - st) * S;
                        T vr[M], vi[M], yr[EM], yi[EM];
                        const T tau = p[0];
#pragma unroll
                        for (int j = 0; j < M; ++j) { vr[j] = p[2 + 2 * j]; vi[j] = p[3 + 2 * j]; }
                        if constexpr (DENSE) {
#pragma unroll
                            for (int c = 0; c < M; ++c) { yr[c] = p[2 + 2 * M + 2 * c]; yi[c] = p[3 + 2 * M + 2 * c]; }
                        } else {
                            yr[0] = T(0);
                            yi[0] = T(0);
                        }
                        apply_step<T, M, R, EM, Q, R, DENSE, false>(wr, wi, er, ei, vr, vi, tau, yr, yi, ch,
                                                                    k - 1 - M, lo, lane, sgr, sgi, dummy_r,
                                                                    dummy_i);
                    }
                });
            }
        }

        // ---- produce this tile's reflectors: steps hi-1 .. lo ------------------
        tri_phase<T, M, DENSE, false>(n, lo, hi, lane, H, ldh, sgr, sgi, rf, tstride, Y, lds_rs, wr, wi, er, ei, singular,
                               nonfinite);

        // this tile's reflector stores complete before the next tile loads them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }

    finish_shift<T, M, DENSE>(n, lane, it.Rtop, Y, lds_rs, it.status, singular, nonfinite);
}

template <typename T, int M, bool DENSE>
__global__ __launch_bounds__(64, 2) void sweep_kernel(SweepArgs<T> a)
{
    __shared__ T lds[sweep_lds_elems<T, M, DENSE>()];
    const int item = blockIdx.x;
    if (item >= (a.dcount ? *a.dcount : a.count)) return;
    const int sid = a.list ? a.list[item] : item;
    SweepItem<T> it;
    it.n = a.n;
    it.H = a.H;
    it.ldh = a.ldh;
    it.sgr = (T)a.shifts[2 * sid];
    it.sgi = (T)a.shifts[2 * sid + 1];
    it.rf = a.refl + (int64_t)sid * a.refl_stride;
    it.Y = a.Y + (int64_t)sid * a.y_stride;
    it.E = DENSE ? a.E + (int64_t)sid * a.e_stride : nullptr;
    it.Rtop = a.Rtop;
    it.status = a.status + sid;
    sweep_body<T, M, DENSE>(it, lds, lds + SweepShape<T, M, DENSE>::CH);
}

}  // namespace shs
