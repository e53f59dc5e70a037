// Q* pass: X = P_{n-1} ... P_1 P_0 [Y; 0] (or ... P_0 y for a dense y).
//
// Section 3.3 forms each solution as x = Q_sigma^*(:, 1:m) y with y the
// small triangular solve; with Q_sigma^* = P_{n-1} ... P_0 kept as the stored
// reflectors of the sweep, applying them to [Y; 0] from P_0 upward gives
// exactly that product without forming Q_sigma.  Every P_k is Hermitian and
// acts on rows k-m .. k only, so the pass walks down the rows with an
// (m+1)-row window: step k applies P_k, then row k-m is final and leaves.
//
// GPU mapping: one lane per (shift, right-hand-side column); a wave holds
// 64/m shifts.  The window again rotates through registers (logical row
// k-m+j in slot (j + k) mod (m+1)).  Accumulation is FP64 whatever the
// precision of the reflectors.
#pragma once

#include <utility>

#include "common.hpp"
#include "sweep.hpp"

namespace shs {

template <typename T>
struct QstarArgs {
    int n, count;
    const int32_t *list;         // work item -> shift id (nullptr = identity)
    const T *refl;               // reflector store of the sweep that produced Y
    int64_t refl_stride;
    int tile_rows;               // rows per tile of that sweep
    int64_t tile_stride;         // elements per tile in the store
    int slot;                    // elements per slot
    const T *Y;                  // structured: m x m (ld m); dense: n x m (ld n)
    int64_t y_stride;
    double *X;                   // n x (s m) complex, ld ldx; column sid*m + c
    int64_t ldx;
    int accumulate;              // 0: X = D, 1: X += scale[sid] * D
    const double *scale;         // per shift id, or nullptr (= 1)
    const int *dcount;           // if set, the number of work items is read here (count is an upper bound)
};

// One lane's share of the Q* pass: column c of one shift.  rf is the
// shift's reflector store (tile_rows, tile_stride, slot describe its layout),
// X points at column c of the shift's output block.
template <typename T, int M, bool DENSE_IN>
__device__ __forceinline__ void qstar_body(int n, bool active, int c, const T *rf, int tile_rows,
                                           int64_t tile_stride, int slot, const T *Y, double *X,
                                           int accumulate, double sc)
{
    constexpr int NP = M + 1;
    auto slot_ptr = [&](int k) -> const T * {
        const int t = k / tile_rows;
        return rf + (int64_t)t * tile_stride + (int64_t)(k - t * tile_rows) * slot;
    };
    auto input_row = [&](int i, double &xr, double &xi) {
        xr = 0.0;
        xi = 0.0;
        if (!active || i >= n) return;
        if constexpr (DENSE_IN) {
            xr = (double)Y[2 * ((int64_t)c * n + i)];
            xi = (double)Y[2 * ((int64_t)c * n + i) + 1];
        } else {
            if (i < M) {
                xr = (double)Y[2 * (c * M + i)];
                xi = (double)Y[2 * (c * M + i) + 1];
            }
        }
    };

    double yr[NP], yi[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) { yr[j] = 0.0; yi[j] = 0.0; }
    input_row(0, yr[M], yi[M]);   // phase 0: logical j in slot j; row 0 is logical m

    double vr[M], vi[M], tau = 0.0;
    double nvr[M], nvi[M], ntau = 0.0;
    auto load = [&](int k, double (&lr)[M], double (&li)[M], double &lt) {
        if (active && k < n) {
            const T *p = slot_ptr(k);
            lt = (double)p[0];
#pragma unroll
            for (int j = 0; j < M; ++j) { lr[j] = (double)p[2 + 2 * j]; li[j] = (double)p[3 + 2 * j]; }
        } else {
            lt = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) { lr[j] = 0.0; li[j] = 0.0; }
        }
    };
    load(0, nvr, nvi, ntau);

    const int k_last = n - 1 + M;   // steps k >= n only flush the window
    for (int kg = 0; kg <= k_last; kg += NP) {
        static_for<NP>([&](auto qc) {
            constexpr int Q = decltype(qc)::value;   // k mod (m+1)
            const int k = kg + Q;
            if (k <= k_last) {
#pragma unroll
                for (int j = 0; j < M; ++j) { vr[j] = nvr[j]; vi[j] = nvi[j]; }
                tau = ntau;
                load(k + 1, nvr, nvi, ntau);
                if (k < n) {
                    // d = v^* y over rows k-m .. k (v_m = 1)
                    constexpr int pm = (M + Q) % NP;
                    double dr = yr[pm], di = yi[pm];
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        const int p = (j + Q) % NP;
                        // conj(v_j) * y_j
                        dr = fma(vr[j], yr[p], fma(vi[j], yi[p], dr));
                        di = fma(vr[j], yi[p], fma(-vi[j], yr[p], di));
                    }
                    const double tr = tau * dr, ti = tau * di;
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        const int p = (j + Q) % NP;
                        // y_j -= t v_j
                        yr[p] = fma(-tr, vr[j], fma(ti, vi[j], yr[p]));
                        yi[p] = fma(-tr, vi[j], fma(-ti, vr[j], yi[p]));
                    }
                    yr[pm] -= tr;
                    yi[pm] -= ti;
                }
                // row k-m (logical 0, slot Q) is final
                const int row = k - M;
                if (active && row >= 0 && row < n) {
                    double *px = X + 2 * (int64_t)row;
                    if (accumulate) {
                        px[0] += sc * yr[Q];
                        px[1] += sc * yi[Q];
                    } else {
                        px[0] = yr[Q];
                        px[1] = yi[Q];
                    }
                }
                // row k+1 enters in the freed slot
                input_row(k + 1, yr[Q], yi[Q]);
            }
        });
    }
}

template <typename T, int M, bool DENSE_IN>
__global__ __launch_bounds__(64) void qstar_kernel(QstarArgs<T> a)
{
    constexpr int SPW = kWave / M;
    const int lane = threadIdx.x;
    const int sw = lane / M, c = lane % M;
    const int item = blockIdx.x * SPW + sw;
    const int count = a.dcount ? *a.dcount : a.count;
    const bool active = (sw < SPW) && (item < count);
    const int sid = active ? (a.list ? a.list[item] : item) : 0;
    const T *rf = a.refl + (int64_t)sid * a.refl_stride;
    const T *Y = a.Y + (int64_t)sid * a.y_stride;
    double *X = a.X + ((int64_t)sid * M + c) * a.ldx * 2;
    const double sc = (a.accumulate && a.scale) ? a.scale[sid] : 1.0;
    qstar_body<T, M, DENSE_IN>(a.n, active, c, rf, a.tile_rows, a.tile_stride, a.slot, Y, X, a.accumulate, sc);
}

// Structured right-hand side ([Y; 0], Y m x m), spw shifts per wavefront
// (spw a power of two, spw m <= 64): lanes q m + c, c < m, own column c of
// the wave's shift q as above, while the whole wave stages the shifts'
// reflectors through LDS in chunks of whole phase groups (coalesced loads,
// the next chunk in flight while the current one is used), so the serial
// chain of n steps does not wait on memory.  spw is chosen by the caller to
// give about one wave per SIMD.  The inner product v^* y is summed in two
// interleaved partial sums to halve its dependence chain.  It writes X
// (no accumulation: the mixed path's corrections use qstar_kernel).
constexpr int kQstarLds = 1536;   // LDS elements of one chunk (all shifts)

// Step k (phase Q = k mod (m+1)) of one lane of qstar_wave_kernel: apply
// P_k (its slot at pv) to the window, emit row k-m into X and let row k+1
// of [Y; 0] in.  GUARD handles the steps near the ends: k >= n only flushes,
// rows outside 0 .. n-1 are not stored, rows below m come from Y.
template <typename T, int M, int Q, bool GUARD>
__device__ __forceinline__ void qstar_wave_step(int k, int n, const T *pv, const T *yl, double *X, double (&yr)[M + 1],
                                                double (&yi)[M + 1])
{
    constexpr int NP = M + 1;
    if (!GUARD || k < n) {
        const double tau = (double)pv[0];
        double vr[M], vi[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            vr[j] = (double)pv[2 + 2 * j];
            vi[j] = (double)pv[3 + 2 * j];
        }
        // d = v^* y over rows k-m .. k (v_m = 1)
        constexpr int pm = (M + Q) % NP;
        double dr0 = yr[pm], di0 = yi[pm], dr1 = 0.0, di1 = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int p = (j + Q) % NP;
            if (j & 1) {
                dr1 = fma(vr[j], yr[p], fma(vi[j], yi[p], dr1));
                di1 = fma(vr[j], yi[p], fma(-vi[j], yr[p], di1));
            } else {
                dr0 = fma(vr[j], yr[p], fma(vi[j], yi[p], dr0));
                di0 = fma(vr[j], yi[p], fma(-vi[j], yr[p], di0));
            }
        }
        const double tr = tau * (dr0 + dr1), ti = tau * (di0 + di1);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int p = (j + Q) % NP;
            yr[p] = fma(-tr, vr[j], fma(ti, vi[j], yr[p]));
            yi[p] = fma(-tr, vi[j], fma(-ti, vr[j], yi[p]));
        }
        yr[pm] -= tr;
        yi[pm] -= ti;
    }
    // row k-m (logical 0, slot Q) is final
    const int row = k - M;
    if (!GUARD || (row >= 0 && row < n)) {
        double *px = X + 2 * (int64_t)row;
        px[0] = yr[Q];
        px[1] = yi[Q];
    }
    // row k+1 enters in the freed slot: [Y; 0]
    if constexpr (GUARD) {
        const int i = k + 1;
        const bool in = i < M && i < n;
        yr[Q] = in ? (double)yl[2 * (in ? i : 0)] : 0.0;
        yi[Q] = in ? (double)yl[2 * (in ? i : 0) + 1] : 0.0;
    } else {
        yr[Q] = 0.0;
        yi[Q] = 0.0;
    }
}

template <typename T, int M>
__global__ __launch_bounds__(64) void qstar_wave_kernel(QstarArgs<T> a, int spw)
{
    constexpr int NP = M + 1;
    constexpr int S = slot_elems(M, false);
    constexpr int CE = kQstarLds;
    constexpr int PL = CE / kWave;
    static_assert(CE % kWave == 0 && CE >= S * NP + 1, "chunk");
    __shared__ T lds_ch[CE];
    __shared__ T lds_y[kWave * 2 * M];   // every shift's Y (spw m <= 64)
    const int lane = threadIdx.x;
    const int n = a.n;
    // steps per chunk (at most a tile, so a chunk spans two tiles at most)
    // and LDS stride per shift (odd: the shifts' reads fall in different banks)
    const int CS = NP * (min((CE / spw - 1) / S, a.tile_rows) / NP);
    const int RS = CS * S + 1;
    const int gl = kWave / spw;                  // lanes loading one shift's chunk
    const int lq = lane / gl, ll = lane % gl;    // loader: shift, lane within
    const int q = lane / M, c = lane % M;        // compute: shift, column
    const int item = blockIdx.x * spw + q;
    const int count = a.dcount ? *a.dcount : a.count;
    if (blockIdx.x * spw >= count) return;   // uniform: no shift of this wave is listed
    const bool active = q < spw && item < count;
    const int litem = blockIdx.x * spw + lq;
    const bool lact = litem < count;
    const int sid = active ? (a.list ? a.list[item] : item) : 0;
    const int lsid = lact ? (a.list ? a.list[litem] : litem) : 0;
    const T *rf = a.refl + (int64_t)lsid * a.refl_stride;
    double *X = a.X + ((int64_t)sid * M + c) * a.ldx * 2;
    const int ce_elems = CS * S;   // elements of one shift's chunk
    const int tt = a.tile_rows;
    T pre[PL];
    // steps past n-1 are read from step n-1 and never used
    auto fetch = [&](int cb) {
        const int t0 = cb / tt, kb = (t0 + 1) * tt;   // the chunk spans tiles t0, t0 + 1
#pragma unroll
        for (int e = 0; e < PL; ++e) {
            const int idx0 = e * gl + ll;
            const int idx = idx0 < ce_elems ? idx0 : ce_elems - 1;
            const int ks = idx / S, el = idx - ks * S;
            const int k = min(cb + ks, n - 1);
            const int t = k < kb ? t0 : t0 + 1;
            pre[e] = rf[(int64_t)t * a.tile_stride + (int64_t)(k - t * tt) * S + el];
        }
    };
    // Y of every shift into LDS, so the rows entering in the first m steps
    // are no memory loads (a wait for one would also wait for the stores of
    // X and the chunk in flight)
    {
        const T *ys = a.Y + (int64_t)lsid * a.y_stride;
        for (int e = ll; e < 2 * M * M; e += gl) lds_y[lq * 2 * M * M + e] = ys[e];
    }
    __syncthreads();
    // Y(:, c) of this lane's shift (idle lanes, q >= spw, point at shift 0's)
    const T *yl = lds_y + (q < spw ? q : 0) * 2 * M * M + 2 * c * M;
    double yr[NP], yi[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) { yr[j] = 0.0; yi[j] = 0.0; }
    // phase 0: logical j in slot j; row 0 is logical m
    yr[M] = (double)yl[0];
    yi[M] = (double)yl[1];
    const int k_last = n - 1 + M;   // steps k >= n only flush the window
    fetch(0);
    for (int cb = 0; cb <= k_last; cb += CS) {
        __syncthreads();            // previous chunk fully read
#pragma unroll
        for (int e = 0; e < PL; ++e) {
            const int idx = e * gl + ll;
            if (idx < ce_elems) lds_ch[lq * RS + idx] = pre[e];
        }
        __syncthreads();
        if (cb + CS < n) fetch(cb + CS);
        if (active) {
            const T *base = lds_ch + q * RS;
            const int ce = min(k_last + 1, cb + CS);
            for (int kg = cb; kg < ce; kg += NP) {
                if (kg >= M && kg + NP <= n && kg + NP <= ce) {
                    // a whole phase group inside the matrix: no guards, so the
                    // group is one straight block (the next step's LDS reads
                    // can go ahead of this step's arithmetic)
                    static_for<NP>([&](auto qc) {
                        constexpr int Q = decltype(qc)::value;   // k mod (m+1)
                        qstar_wave_step<T, M, Q, false>(kg + Q, n, base + (kg + Q - cb) * S, yl, X, yr, yi);
                    });
                } else {
                    static_for<NP>([&](auto qc) {
                        constexpr int Q = decltype(qc)::value;
                        if (kg + Q < ce)
                            qstar_wave_step<T, M, Q, true>(kg + Q, n, base + (kg + Q - cb) * S, yl, X, yr, yi);
                    });
                }
            }
        }
    }
}

// Shifts per wave for count shifts at m: about one wave per SIMD (1024 of
// them), as many shifts as the lanes and a chunk of at least one phase
// group per shift allow.
inline int qstar_spw(int64_t count, int m)
{
    const int S = slot_elems(m, false);
    int spw = 1;
    while (spw * 2 * m <= kWave && (kQstarLds / (spw * 2) - 1) / S >= m + 1 && count > (int64_t)spw * 1024) spw *= 2;
    return spw;
}

}  // namespace shs

namespace shs {

// Dense y (the correction solves and the transposed systems): X (+)= P_{n-1}
// ... P_0 y, y the n x m result of a dense-right-hand-side sweep.  The same
// wave organisation as qstar_wave_kernel: spw shifts per wavefront, lane
// q m + c owns column c of shift q, the reflector slots staged through LDS in
// chunks of whole phase groups.  The row entering at step k is y_{k+1},
// which the dense sweep stored in slot k+1, so a chunk of steps cb .. cb+CS-1
// stages slots cb .. cb+CS (one more than it applies).  With accumulate set,
// X += scale[sid] * (the product).
template <typename T, int M>
__global__ __launch_bounds__(64) void qstar_wave_dense_kernel(QstarArgs<T> a, int spw)
{
    constexpr int NP = M + 1;
    constexpr int S = slot_elems(M, true);
    constexpr int CE = kQstarLds;
    constexpr int PL = CE / kWave;
    static_assert(CE % kWave == 0 && CE >= S * (NP + 1) + 1, "chunk");
    __shared__ T lds_ch[CE];
    const int lane = threadIdx.x;
    const int n = a.n;
    // steps per chunk (at most a tile, so a chunk spans two tiles at most)
    // and LDS stride per shift (odd: the shifts' reads fall in different banks)
    const int CS = NP * (min((CE / spw - 1) / S - 1, a.tile_rows) / NP);
    const int RS = (CS + 1) * S + 1;
    const int gl = kWave / spw;                  // lanes loading one shift's chunk
    const int lq = lane / gl, ll = lane % gl;    // loader: shift, lane within
    const int q = lane / M, c = lane % M;        // compute: shift, column
    const int item = blockIdx.x * spw + q;
    const int count = a.dcount ? *a.dcount : a.count;
    if (blockIdx.x * spw >= count) return;   // uniform: no shift of this wave is listed
    const bool active = q < spw && item < count;
    const int litem = blockIdx.x * spw + lq;
    const bool lact = litem < count;
    const int sid = active ? (a.list ? a.list[item] : item) : 0;
    const int lsid = lact ? (a.list ? a.list[litem] : litem) : 0;
    const T *rf = a.refl + (int64_t)lsid * a.refl_stride;
    double *X = a.X + ((int64_t)sid * M + c) * a.ldx * 2;
    const double sc = (a.accumulate && a.scale) ? a.scale[sid] : 1.0;
    const int ce_elems = (CS + 1) * S;   // elements of one shift's chunk
    const int tt = a.tile_rows;
    T pre[PL];
    // slots past n-1 are read from slot n-1 and never used
    auto fetch = [&](int cb) {
        const int t0 = cb / tt, kb = (t0 + 1) * tt;   // the chunk spans tiles t0, t0 + 1
#pragma unroll
        for (int e = 0; e < PL; ++e) {
            const int idx0 = e * gl + ll;
            const int idx = idx0 < ce_elems ? idx0 : ce_elems - 1;
            const int ks = idx / S, el = idx - ks * S;
            const int k = min(cb + ks, n - 1);
            const int t = k < kb ? t0 : t0 + 1;
            pre[e] = rf[(int64_t)t * a.tile_stride + (int64_t)(k - t * tt) * S + el];
        }
    };
    double yr[NP], yi[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) { yr[j] = 0.0; yi[j] = 0.0; }
    const int k_last = n - 1 + M;   // steps k >= n only flush the window
    fetch(0);
    for (int cb = 0; cb <= k_last; cb += CS) {
        __syncthreads();            // previous chunk fully read
#pragma unroll
        for (int e = 0; e < PL; ++e) {
            const int idx = e * gl + ll;
            if (idx < ce_elems) lds_ch[lq * RS + idx] = pre[e];
        }
        __syncthreads();
        if (cb + CS < n) fetch(cb + CS);
        if (active) {
            const T *base = lds_ch + q * RS;
            if (cb == 0) {
                // phase 0: row 0 (y_0, in slot 0) is logical m
                yr[M] = (double)base[2 + 2 * M + 2 * c];
                yi[M] = (double)base[3 + 2 * M + 2 * c];
            }
            const int ce = min(k_last + 1, cb + CS);
            for (int kg = cb; kg < ce; kg += NP) {
                static_for<NP>([&](auto qc) {
                    constexpr int Q = decltype(qc)::value;   // k mod (m+1)
                    const int k = kg + Q;
                    if (k < ce) {
                        const T *pv = base + (k - cb) * S;
                        if (k < n) {
                            const double tau = (double)pv[0];
                            double vr[M], vi[M];
#pragma unroll
                            for (int j = 0; j < M; ++j) {
                                vr[j] = (double)pv[2 + 2 * j];
                                vi[j] = (double)pv[3 + 2 * j];
                            }
                            constexpr int pm = (M + Q) % NP;
                            double dr0 = yr[pm], di0 = yi[pm], dr1 = 0.0, di1 = 0.0;
#pragma unroll
                            for (int j = 0; j < M; ++j) {
                                const int p = (j + Q) % NP;
                                if (j & 1) {
                                    dr1 = fma(vr[j], yr[p], fma(vi[j], yi[p], dr1));
                                    di1 = fma(vr[j], yi[p], fma(-vi[j], yr[p], di1));
                                } else {
                                    dr0 = fma(vr[j], yr[p], fma(vi[j], yi[p], dr0));
                                    di0 = fma(vr[j], yi[p], fma(-vi[j], yr[p], di0));
                                }
                            }
                            const double tr = tau * (dr0 + dr1), ti = tau * (di0 + di1);
#pragma unroll
                            for (int j = 0; j < M; ++j) {
                                const int p = (j + Q) % NP;
                                yr[p] = fma(-tr, vr[j], fma(ti, vi[j], yr[p]));
                                yi[p] = fma(-tr, vi[j], fma(-ti, vr[j], yi[p]));
                            }
                            yr[pm] -= tr;
                            yi[pm] -= ti;
                        }
                        // row k-m (logical 0, slot Q) is final
                        const int row = k - M;
                        if (row >= 0 && row < n) {
                            double *px = X + 2 * (int64_t)row;
                            if (a.accumulate) {
                                px[0] += sc * yr[Q];
                                px[1] += sc * yi[Q];
                            } else {
                                px[0] = yr[Q];
                                px[1] = yi[Q];
                            }
                        }
                        // row k+1 enters in the freed slot: y_{k+1}, from slot k+1
                        const bool in = k + 1 < n;
                        const T *pn = base + (in ? k + 1 - cb : 0) * S;
                        yr[Q] = in ? (double)pn[2 + 2 * M + 2 * c] : 0.0;
                        yi[Q] = in ? (double)pn[3 + 2 * M + 2 * c] : 0.0;
                    }
                });
            }
        }
    }
}

// Shifts per wave of the dense Q* pass: about one wave per SIMD, as many
// shifts as the lanes and a chunk of at least two phase groups per shift allow.
inline int qstar_dense_spw(int64_t count, int m)
{
    const int S = slot_elems(m, true);
    int spw = 1;
    while (spw * 2 * m <= kWave && (kQstarLds / (spw * 2) - 1) / S - 1 >= 2 * (m + 1) && count > (int64_t)spw * 1024)
        spw *= 2;
    return spw;
}

}  // namespace shs
