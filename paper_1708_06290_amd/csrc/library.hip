// C-ABI entry points of the shiftsolve library (declared in shiftsolve.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "shiftsolve.h"
#include "handle.hpp"
#include "blocked.hpp"
#include "gemm.hpp"
#include "kernels.hpp"
#include "reduce.hpp"
#include "residual.hpp"

using namespace shs;


namespace {

template <typename T>
hipError_t dmalloc(T **p, size_t count, size_t *acc)
{
    hipError_t e = hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1));
    if (e == hipSuccess && acc) *acc += sizeof(T) * std::max<size_t>(count, 1);
    return e;
}

void free_handle(shs_handle *h)
{
    if (!h) return;
    for (hipEvent_t ev : h->pool) hipEventDestroy(ev);
    hipFree(h->H);
    hipFree(h->H32);
    hipFree(h->Bw);
    hipFree(h->Rtop);
    hipFree(h->rcolmax);
    hipFree(h->Ct);
    hipFree(h->V);
    hipFree(h->tauv);
    hipFree(h->sgn);
    hipFree(h->offrow);
    hipFree(h->diag);
    hipFree(h->dstats);
    hipFree(h->Ht);
    hipFree(h->ht_offrow);
    hipFree(h->ht_diag);
    if (h->ht_ready) hipEventDestroy(h->ht_ready);
    delete h;
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Records an event pair around one phase when timing is enabled.
struct PhaseScope {
    shs_handle *h;
    hipStream_t st;
    int idx = -1;
    PhaseScope(shs_handle *h_, int phase, int64_t shifts, hipStream_t st_) : h(h_), st(st_)
    {
        if (!h->timing) return;
        const size_t need = 2 * (h->marks.size() + 1);
        while (h->pool.size() < need) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return;
            h->pool.push_back(ev);
        }
        shs_handle::Mark mk{phase, shifts, h->pool[2 * h->marks.size()], h->pool[2 * h->marks.size() + 1]};
        hipEventRecord(mk.a, st);
        idx = (int)h->marks.size();
        h->marks.push_back(mk);
    }
    // closes the phase early (the destructor then does nothing)
    void end()
    {
        if (idx >= 0) hipEventRecord(h->marks[idx].b, st);
        idx = -1;
    }
    ~PhaseScope() { end(); }
};

// start row of reflector idx (0..m-1: QR of B, j; m..: m-Hessenberg column j -> j + m)
inline int64_t refl_start(int64_t m, int64_t idx) { return idx < m ? idx : (idx - m) + m; }

// Apply reflector (v, tau) on rows [r0, r0 + L) from the left to columns
// [c0, c1) of A and from the right to columns [r0, r0 + L) of the first
// `rows` rows of A (two-sided), and from the right to Ct.
hipError_t two_sided(shs_handle *h, double *A, int64_t lda, int64_t L, int64_t r0, int64_t c0,
                     const double *v, const double *tau, double *part, hipStream_t st)
{
    const int64_t n = h->n;
    const int nchunks = (int)cdiv(L, kRightChunk);
    if (n - c0 > 0)
        hipLaunchKernelGGL(left_update_kernel, dim3((unsigned)(n - c0)), dim3(256), 0, st, (int)L, (int)r0,
                           (int)c0, A, lda, v, tau);
    hipLaunchKernelGGL(right_dot_kernel, dim3(cdiv(n, 256), nchunks), dim3(256), 0, st, (int)n, (int)L,
                       (int)r0, (const double *)A, lda, v, tau, part);
    hipLaunchKernelGGL(right_update_kernel, dim3(cdiv(n, 256), nchunks), dim3(256), 0, st, (int)n, (int)L,
                       (int)r0, A, lda, v, tau, (const double *)part, nchunks);
    if (h->p > 0) {
        hipLaunchKernelGGL(right_dot_kernel, dim3(cdiv(h->p, 256), nchunks), dim3(256), 0, st, (int)h->p,
                           (int)L, (int)r0, (const double *)h->Ct, h->ldct, v, tau, part);
        hipLaunchKernelGGL(right_update_kernel, dim3(cdiv(h->p, 256), nchunks), dim3(256), 0, st, (int)h->p,
                           (int)L, (int)r0, h->Ct, h->ldct, v, tau, (const double *)part, nchunks);
    }
    return hipGetLastError();
}

struct Geo {
    SweepGeometry g;
    int64_t stride;   // elements per shift in the reflector store
};

bool geo(bool fp32, int64_t n, int64_t m, bool dense, Geo *out)
{
    if (!sweep_geometry(fp32, (int)m, dense, &out->g)) return false;
    out->stride = out->g.refl_stride((int)n);
    return true;
}

// Workspace layout (byte offsets, each 256-byte aligned).
struct Layout {
    size_t refl64 = 0, y64 = 0, x = 0, resmax = 0, xmax = 0, list = 0;
    size_t refl32 = 0, y32 = 0, e32 = 0, yd32 = 0, res = 0, scale = 0, eta_prev = 0, status2 = 0;
    size_t list2 = 0, fblist = 0, cnt = 0;   // mixed mode: device-side shift lists and their counts
    // blocked FP64 sweep (FP64 mode): carried columns, block transforms
    bool blocked = false;
    size_t zb = 0, bm = 0, m2 = 0, m2p = 0, m2q = 0;
    size_t xt = 0;   // packed solutions for the residual
    int64_t blk_rows = 0, blk_cols = 0;
    // blocked FP32 sweeps of the mixed mode (structured; dense corrections
    // when blk32_dense): their carried columns, block transforms and
    // carried matrices, and the reflector-store stride per shift
    size_t z32 = 0, bm32 = 0, m2a = 0, m2b = 0, m2c = 0;
    int64_t blk32_rows = 0, refl32_stride = 0;
    bool blk32_dense = false;
    size_t total = 0;
};

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// Columns of the carried-column array for count shifts of w real columns:
// whole 128-column tiles of the update, and a whole number of shifts, so
// that every shift a tile touches (padding ones included) has its columns
// and its carried matrix inside the buffers (w = 48 needs multiples of 384).
inline int64_t blk_ncols(int64_t w, int64_t count)
{
    int64_t unit = 128;
    while (unit % w != 0) unit += 128;
    return (w * count + unit - 1) / unit * unit;
}

// Row tiles per update group of the blocked FP64 sweep.
constexpr int kBlkGroup = 4;

bool layout(const shs_handle *h, int64_t s, int mode, int outputs, Layout *L)
{
    const int64_t n = h->n, m = h->m;
    Geo g64, g32s, g32d;
    if (!geo(false, n, m, false, &g64)) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += al(bytes); return o; };
    L->refl64 = take(sizeof(double) * g64.stride * s);
    L->y64 = take(sizeof(double) * 2 * m * m * s);
    L->x = (outputs & SHS_OUT_X) ? 0 : take(sizeof(double) * 2 * n * m * s);
    L->resmax = take(sizeof(unsigned long long) * m * s);
    L->xmax = take(sizeof(unsigned long long) * m * s);
    L->list = take(sizeof(int32_t) * s);
    L->status2 = take(sizeof(int32_t) * s);
    L->xt = take(sizeof(double) * residual_pack_rows(n) * residual_pack_ld(m * s));
    if (mode == SHS_MODE_FP32_REFINE) {
        L->list2 = take(sizeof(int32_t) * s);
        L->fblist = take(sizeof(int32_t) * s);
        L->cnt = take(sizeof(int) * 4);
    }
    // the mixed form's refinement buffers and the blocked FP64 sweep's
    // buffers (its fallback) are never live together: they share one region
    const size_t region = off;
    size_t end_blk = off, end_mix = off;
    {
        int tr = 0, w = 0;
        if (!blk_geometry(false, (int)m, false, &tr, &w)) return false;
        L->blocked = true;
        L->blk_cols = blk_ncols(w, s);
        // rows of the block transforms, up to whole 16-row chunks
        L->blk_rows = (kBlkGroup * tr + m + 15) / 16 * 16;
        L->zb = take(sizeof(double) * n * L->blk_cols);
        L->bm = take(sizeof(double) * L->blk_rows * L->blk_cols);
        L->m2 = take(sizeof(double) * (L->blk_cols / w) * w * w);
        L->m2p = take(sizeof(double) * (L->blk_cols / w) * w * w);
        L->m2q = take(sizeof(double) * (L->blk_cols / w) * w * w);
        end_blk = off;
    }
    if (mode == SHS_MODE_FP32_REFINE) {
        off = region;
        if (!geo(true, n, m, false, &g32s) || !geo(true, n, m, true, &g32d)) return false;
        int trs = 0, ws = 0, trd = 0, wd = 0;
        if (!blk_geometry(true, (int)m, false, &trs, &ws)) return false;
        L->blk32_dense = blk_geometry(true, (int)m, true, &trd, &wd);
        const int64_t wmax = std::max(ws, wd);
        const int64_t cols = std::max(blk_ncols(ws, s), L->blk32_dense ? blk_ncols(wd, s) : 0);
        const int64_t st_s = (n + trs - 1) / trs * refl_tile_stride<float>(trs, slot_elems((int)m, false));
        const int64_t st_d = L->blk32_dense
                                 ? (n + trd - 1) / trd * refl_tile_stride<float>(trd, slot_elems((int)m, true))
                                 : g32d.stride;
        L->refl32_stride = std::max(st_s, st_d);
        L->refl32 = take(sizeof(float) * L->refl32_stride * s);
        L->blk32_rows = (kBlkGroup * std::max(trs, trd) + m + 15) / 16 * 16;
        L->z32 = take(sizeof(float) * n * cols);
        L->bm32 = take(sizeof(float) * L->blk32_rows * cols);
        L->m2a = take(sizeof(float) * cols * wmax);
        L->m2b = take(sizeof(float) * cols * wmax);
        L->m2c = take(sizeof(float) * cols * wmax);
        L->y32 = take(sizeof(float) * 2 * m * m * s);
        L->e32 = take(sizeof(float) * 2 * n * m * s);
        L->yd32 = take(sizeof(float) * 2 * n * m * s);
        L->res = take(sizeof(double) * 2 * n * m * s);
        L->scale = take(sizeof(double) * s);
        L->eta_prev = take(sizeof(double) * s);
        end_mix = off;
    }
    L->total = std::max(end_blk, end_mix);
    return true;
}

template <typename T>
inline T *at(void *base, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }

// E32(:, sid*m + c) = Res(:, sid*m + c) / scale[sid], scale = 2^ceil(log2(max |Res_sid|)),
// for the listed shifts (item = blockIdx.x < *dcount).
__global__ __launch_bounds__(256) void scale_residual_kernel(int n, int m, const int *dcount, const int32_t *list,
                                                             const double *Res, const unsigned long long *resmax,
                                                             double *scale, float *E32)
{
    const int item = blockIdx.x;
    if (item >= *dcount) return;
    const int sid = list[item];
    double mx = 0.0;
    for (int c = 0; c < m; ++c) {
        const double v = __longlong_as_double((long long)resmax[(int64_t)sid * m + c]);
        mx = v > mx ? v : mx;
    }
    const double sc = mx > 0.0 ? exp2(ceil(log2(mx))) : 1.0;
    if (blockIdx.y == 0 && threadIdx.x == 0) scale[sid] = sc;
    const double inv = 1.0 / sc;
    const int64_t total = (int64_t)n * m;
    for (int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.y * 256) {
        const int64_t c = idx / n, i = idx % n;
        const double *pr = Res + (((int64_t)sid * m + c) * n + i) * 2;
        float *pe = E32 + ((int64_t)sid * n * m + c * n + i) * 2;
        pe[0] = (float)(pr[0] * inv);
        pe[1] = (float)(pr[1] * inv);
    }
}

// Mixed mode, device-side bookkeeping (no host synchronisation inside a
// solve).  cnt[0] and cnt[1] are the lengths of the two alternating lists of
// shifts still being refined, cnt[2] that of the fallback list; stats (if
// set, timing only) counts correction rounds, fallback shifts and the
// shift-solves of the correction sweeps.
__global__ void mixed_init_kernel(int s, int32_t *list, double *eta_prev, int *cnt, long long *stats)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < s) {
        list[i] = i;
        eta_prev[i] = __longlong_as_double(0x7ff0000000000000LL);   // +inf
    }
    if (i == 0) {
        cnt[0] = s;
        cnt[1] = 0;
        cnt[2] = 0;
        if (stats) stats[0] = stats[1] = stats[2] = 0;
    }
}

// After the residual of refinement round `it`: every listed shift with
// eta <= tol is done (status OK); one whose eta is NaN, did not at least
// halve since the previous round, or has used max_iter corrections goes to
// the fallback list; the others go to the next list.  One workgroup keeps
// both lists in the order of the input list (block-wide prefix sums).
__global__ __launch_bounds__(1024) void mixed_select_kernel(int it, int max_iter, double tol, const int32_t *in,
                                                            const int *cin, int32_t *out, int *cout, int32_t *fb,
                                                            int *cfb, const double *eta, double *eta_prev,
                                                            int32_t *status, long long *stats)
{
    __shared__ int sn[1024], sf[1024];
    __shared__ int base_n, base_f;
    const int t = threadIdx.x;
    const int count = *cin;
    if (t == 0) {
        base_n = 0;
        base_f = *cfb;
    }
    __syncthreads();
    for (int c0 = 0; c0 < count; c0 += 1024) {
        const int item = c0 + t;
        int kind = 0;   // 0 done or idle, 1 next, 2 fallback
        int sid = 0;
        if (item < count) {
            sid = in[item];
            const double v = eta[sid];
            if (v <= tol) {
                status[sid] = SHS_STATUS_OK;
            } else if (!(v == v) || it >= max_iter || !(v <= 0.5 * eta_prev[sid])) {
                kind = 2;
            } else {
                eta_prev[sid] = v;
                kind = 1;
            }
        }
        sn[t] = kind == 1;
        sf[t] = kind == 2;
        __syncthreads();
        // inclusive prefix sums (Hillis-Steele)
        for (int d = 1; d < 1024; d <<= 1) {
            const int an = t >= d ? sn[t - d] : 0, af = t >= d ? sf[t - d] : 0;
            __syncthreads();
            sn[t] += an;
            sf[t] += af;
            __syncthreads();
        }
        if (kind == 1) out[base_n + sn[t] - 1] = sid;
        if (kind == 2) fb[base_f + sf[t] - 1] = sid;
        __syncthreads();
        if (t == 0) {
            base_n += sn[1023];
            base_f += sf[1023];
        }
        __syncthreads();
    }
    if (t == 0) {
        *cout = base_n;
        *cfb = base_f;
        if (stats) {
            if (base_n > 0) stats[0] += 1;
            stats[1] = base_f;
            stats[2] += base_n;
        }
    }
}

// Final status of the shifts the FP64 sweep recomputed: its own status if
// not OK (singular, non-finite), else FALLBACK when its eta meets tol and
// NOT_CONVERGED otherwise.
__global__ void mixed_final_kernel(const int *cfb, const int32_t *fb, const int32_t *st64, const double *eta,
                                   double tol, int32_t *status)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= *cfb) return;
    const int sid = fb[i];
    const int st = st64[sid];
    status[sid] = st != SHS_STATUS_OK ? st : (eta[sid] <= tol ? SHS_STATUS_FALLBACK : SHS_STATUS_NOT_CONVERGED);
}

// Buffers of the blocked sweep: carried columns Z (n x ncols), block
// transforms Bm (blk_rows x ncols, row-major), per-shift carried matrices.
template <typename T>
struct BlkBufT {
    T *Zb, *Bm, *M2, *M2p, *M2q;
    int64_t blk_rows;
};
using BlkBuf = BlkBufT<double>;

// Z(:, item W + 2m + c) + i Z(:, item W + 3m + c) = E_sid(:, c) (the dense
// right-hand side of the item's shift, E_sid(i, c) at ((sid m + c) n + i) 2)
// and every other column of the item zero: the bottom tile reads e from Z and
// z from H.  Items past the list (and the padding up to a whole 128 columns)
// are all zero: a 16-column block of the update may hold several items, so
// every column it reads must be finite.
template <typename T>
__global__ __launch_bounds__(256) void blk_dense_init_kernel(int n, int m, int W, int count, const int *dcount,
                                                             const int32_t *list, const T *E, T *Z, int64_t ldz)
{
    const int v = blockIdx.y, q = blockIdx.z;   // item, column within the item
    const int cnt = dcount ? *dcount : count;
    // an item past the list whose 16-column block holds no listed item is
    // never read by a launch that stores results (an empty list: none is)
    if (v >= cnt && (cnt == 0 || (v * W) / 16 > ((cnt * W) - 1) / 16)) return;
    T *z = Z + ((int64_t)v * W + q) * ldz;
    const int c = q - 2 * m;
    const bool re = v < cnt && c >= 0 && c < m, im = v < cnt && c >= m && c < 2 * m;
    const int sid = v < cnt ? (list ? list[v] : v) : 0;
    const T *src = E + ((int64_t)sid * m + (re ? c : c - m)) * n * 2 + (re ? 0 : 1);
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        z[i] = (re || im) ? src[2 * (int64_t)i] : T(0);
}

// Blocked sweep of the listed shifts (FP64 on H, or FP32 on H32 for the
// mixed form): per row tile (bottom to top) the per-shift tile kernel, then
// the all-shift update of the rows above.  With E set, the right-hand side
// is dense (m columns per shift id, laid out as for blk_dense_init_kernel,
// m <= kBlkDenseMaxM) and the matrix is Hm (H, H32 or H's order-reversed
// transpose).  ph: the timing phase of the whole sweep.
template <typename T>
hipError_t sweep_blocked(shs_handle *h, int64_t count, const int32_t *dlist, const int *dcount, const double *shifts,
                         const BlkBufT<T> &B, const SweepArgs<T> &sa, hipStream_t st, const T *E = nullptr,
                         const T *Hm = nullptr, int ph = PH_SWEEP)
{
    const int n = (int)h->n, m = (int)h->m;
    const bool dense = E != nullptr;
    constexpr bool fp32 = sizeof(T) == 4;
    if (!Hm) Hm = fp32 ? (const T *)(const void *)h->H32 : (const T *)(const void *)h->H;
    int tr = 0, w = 0;
    if (!blk_geometry(fp32, m, dense, &tr, &w)) return hipErrorInvalidValue;
    if (count <= 0) return hipSuccess;
    const int ntiles = (n + tr - 1) / tr;
    const int64_t ncols = blk_ncols(w, count);
    if (ncols % 128 != 0 || ncols % w != 0) return hipErrorInvalidValue;
    T *Zb = B.Zb, *Bm = B.Bm, *M2 = B.M2, *M2p = B.M2p, *M2q = B.M2q;
    PhaseScope whole(h, ph, count, st);
    if (dense) {
        hipLaunchKernelGGL(blk_dense_init_kernel<T>, dim3(cdiv(n, 256 * 8), (unsigned)(ncols / w), (unsigned)w),
                           dim3(256), 0, st, n, m, w, (int)count, dcount, dlist, E, Zb, (int64_t)n);
        const hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
    }
    // columns past 2m of each shift, those of the padding shifts and the
    // rows past the bottom tile's K stay zero.  Bm is row-major with row
    // stride ncols.
    hipError_t e = zero_fill(Bm, sizeof(T) * B.blk_rows * ncols, st);
    if (e != hipSuccess) return e;
    e = zero_fill(M2, sizeof(T) * (ncols / w) * w * w, st);
    if (e != hipSuccess) return e;
    e = zero_fill(M2p, sizeof(T) * (ncols / w) * w * w, st);
    if (e != hipSuccess) return e;
    e = zero_fill(M2q, sizeof(T) * (ncols / w) * w * w, st);
    if (e != hipSuccess) return e;
    BlkTriArgsT<T> ta{};
    ta.n = n;
    ta.count = (int)count;
    ta.ntiles = ntiles;
    ta.H = Hm;
    ta.ldh = h->ldh;
    ta.shifts = shifts;
    ta.list = dlist;
    ta.Rtop = h->Rtop;
    ta.refl = sa.refl;
    ta.refl_stride = sa.refl_stride;
    ta.Y = sa.Y;
    ta.y_stride = sa.y_stride;
    ta.status = sa.status;
    ta.Z = Zb;
    ta.ldz = n;
    ta.Bm = Bm;
    ta.ldb = ncols;
    ta.M2 = M2;
    ta.D = kBlkGroup;
    ta.dcount = dcount;
    ZupdArgsT<T> za{};
    za.m = m;
    za.n = n;
    za.ncols = (int)ncols;
    za.count = (int)count;
    za.nr = dense ? m : 0;
    za.H = Hm;
    za.ldh = h->ldh;
    za.Bm = Bm;
    za.ldb = ncols;
    za.M2 = M2;
    za.Z = Zb;
    za.ldz = n;
    za.shifts = shifts;
    za.list = dlist;
    za.dcount = dcount;
    // bottom tile: all rows above it at once (K = n_b + m, no Z yet); then
    // groups of kBlkGroup tiles: after the k-th, the next tile's rows get the
    // group's composite (K = k n_b); after the last, all rows above do
    int k = 0;
    T *m2cur = M2p, *m2nxt = M2q;   // composite M2: read, written
    for (int t = ntiles - 1; t >= 0; --t) {
        const bool bottom = t == ntiles - 1;
        ta.t = t;
        if (!bottom) ++k;
        ta.gk = bottom ? 0 : k;
        ta.M2p = m2cur;
        ta.M2q = m2nxt;
        {
            PhaseScope ps(h, PH_TILE, count, st);
            if (!launch_blk_tri(m, dense, ta, st)) return hipErrorInvalidValue;
        }
        if (h->timing && !dcount) {   // timing state is only touched when enabled (flops: host-known counts only)
            // steps: (16m+4) flops per row above the pivot in the tile; the
            // block transform: n_b reflectors on m columns of length m+1; a
            // group's k-th tile: its older composite rows and M2 times 2m x 2m
            // (a dense right-hand side: the e updates inside the tile, N_blk
            // beside M_blk, and 4m x 4m carried matrices)
            const double nb = std::min(n, t * tr + tr) - t * tr, w2 = (dense ? 4.0 : 2.0) * m;
            double f = ((dense ? 24.0 : 16.0) * m + 4.0) * nb * (nb - 1.0) / 2.0;
            if (t > 0) f += 16.0 * (m + 1) * (dense ? 2 * m : m) * nb;
            if (t > 0 && k >= 2) f += 2.0 * ((k - 1) * tr + w2) * w2 * w2;
            h->tile_flops += f * (double)count;
        }
        if (!bottom) std::swap(m2cur, m2nxt);   // m2cur: composite including tile t
        if (t == 0) break;
        const int lo = t * tr, hi = std::min(n, lo + tr);
        za.lo = lo;
        za.c0 = lo - m;
        if (bottom) {
            za.r0 = 0;
            za.K = hi - lo + m;
            za.has_zin = dense ? 1 : 0;   // a dense right-hand side is carried in Z from the start
            za.Bm = Bm;
            za.M2 = M2;
        } else if (k < kBlkGroup) {
            za.r0 = lo - tr;   // the next tile's rows
            za.K = k * tr;
            za.has_zin = 1;
            za.Bm = Bm + (int64_t)(kBlkGroup - k) * tr * ncols;
            za.M2 = m2cur;
        } else {
            za.r0 = 0;
            za.K = kBlkGroup * tr;
            za.has_zin = 1;
            za.Bm = Bm;
            za.M2 = m2cur;
            k = 0;
        }
        {
            PhaseScope ps(h, PH_UPDATE, count, st);
            if (!launch_zupd(m, za, st)) return hipErrorInvalidValue;
        }
        // H(rows, K columns) times 2m real columns per shift, plus z times a
        // 2m x 2m matrix when carried columns are read
        if (h->timing && !dcount)
            h->update_flops +=
                (2.0 * (za.lo - za.r0) * za.K * (dense ? 4 : 2) * m +
                 (za.has_zin ? 2.0 * (za.lo - za.r0) * 2.0 * m * (dense ? 4 : 2) * m : 0.0)) *
                (double)count;
    }
    return hipGetLastError();
}

// Y_j <- [Y_j b_j, 0, ..., 0] for the m x m result Y_j = R_sigma^{-1} R(0:m,0:m)
// of the sweep (one block per shift; thread i owns row i).
__global__ __launch_bounds__(64) void vec_y_kernel(int m, double *Y, const double *bhat, int64_t ldb)
{
    const int j = blockIdx.x, i = threadIdx.x;
    if (i >= m) return;
    double *Yj = Y + (int64_t)j * 2 * m * m;
    const double *b = bhat + (int64_t)j * ldb * 2;
    double yr = 0.0, yi = 0.0;
    for (int c = 0; c < m; ++c) {
        const double ar = Yj[2 * (c * m + i)], ai = Yj[2 * (c * m + i) + 1];
        yr = fma(ar, b[2 * c], fma(-ai, b[2 * c + 1], yr));
        yi = fma(ar, b[2 * c + 1], fma(ai, b[2 * c], yi));
    }
    Yj[2 * i] = yr;
    Yj[2 * i + 1] = yi;
    for (int c = 1; c < m; ++c) Yj[2 * (c * m + i)] = Yj[2 * (c * m + i) + 1] = 0.0;
}

// FP64 sweep + Q* pass for the listed shifts into X (dcount: the list's
// length on the device, count then an upper bound).
//
// With per-shift directions bhat (m x count complex, ld ldb; list and count
// on the device not allowed), each Y_j becomes [Y_j b_j, 0, ..., 0] before
// the Q* pass, so the shift's first output column is (H - sigma_j I)^{-1} R b_j.
hipError_t solve_fp64(shs_handle *h, int64_t count, const int32_t *dlist, const int *dcount, const double *shifts,
                      void *work, const Layout &L, double *X, int64_t ldx, int32_t *status, hipStream_t st,
                      const double *bhat = nullptr, int64_t ldb = 0)
{
    const int64_t n = h->n, m = h->m;
    Geo g;
    geo(false, n, m, false, &g);
    SweepArgs<double> sa{};
    sa.n = (int)n;
    sa.count = (int)count;
    sa.H = h->H;
    sa.ldh = h->ldh;
    sa.shifts = shifts;
    sa.list = dlist;
    sa.Rtop = h->Rtop;
    sa.refl = at<double>(work, L.refl64);
    sa.refl_stride = g.stride;
    sa.Y = at<double>(work, L.y64);
    sa.y_stride = 2 * m * m;
    sa.status = status;
    sa.dcount = dcount;
    if (L.blocked) {
        const BlkBuf B{at<double>(work, L.zb), at<double>(work, L.bm), at<double>(work, L.m2),
                       at<double>(work, L.m2p), at<double>(work, L.m2q), L.blk_rows};
        hipError_t e = sweep_blocked(h, count, dlist, dcount, shifts, B, sa, st);
        if (e != hipSuccess) return e;
    } else {
        PhaseScope ps(h, PH_SWEEP, count, st);
        if (!launch_sweep((int)m, false, sa, st)) return hipErrorInvalidValue;
    }
    if (bhat) {
        if (dlist || dcount) return hipErrorInvalidValue;
        PhaseScope ps(h, PH_OTHER, count, st);
        hipLaunchKernelGGL(vec_y_kernel, dim3((unsigned)count), dim3(64), 0, st, (int)m, sa.Y, bhat, ldb);
    }
    QstarArgs<double> qa{};
    qa.n = (int)n;
    qa.count = (int)count;
    qa.list = dlist;
    qa.refl = sa.refl;
    qa.refl_stride = g.stride;
    qa.tile_rows = g.g.tile_rows;
    qa.tile_stride = g.g.tile_stride;
    qa.slot = g.g.slot;
    qa.Y = sa.Y;
    qa.y_stride = 2 * m * m;
    qa.X = X;
    qa.ldx = ldx;
    qa.accumulate = 0;
    qa.scale = nullptr;
    qa.dcount = dcount;
    {
        PhaseScope ps(h, PH_QSTAR, count, st);
        if (!launch_qstar((int)m, false, qa, st)) return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- transposed systems (H - sigma I)^T Y = D -----------------------------
// With J the order-reversing permutation, J (H - sigma I)^T J = Ht - sigma I
// where Ht = J H^T J, Ht(i, j) = H(n-1-j, n-1-i), is upper m-Hessenberg again:
// (H - sigma I)^T Y = D  <=>  (Ht - sigma I) (J Y) = J D.  The bottom-up RQ
// sweep of Ht - sigma I with the right-hand side J D is the top-down LQ
// factorisation (H - sigma I)^T = L Q of Section 3.3, with the forward
// substitution for L fused into it, in reversed index order.

// Ht = J H^T J through 64 x 64 LDS tiles: loads along the columns of H,
// stores along the columns of Ht.
__global__ __launch_bounds__(256) void transpose_reverse_kernel(int n, const double *H, int64_t ldh, double *Ht)
{
    __shared__ double t[64][65];
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;   // Ht rows i0.., columns j0..
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // Ht(i, j) = H(n-1-j, n-1-i): rows r = n-1-j of H, columns c = n-1-i
    for (int q = ty; q < 64; q += 4) {
        const int i = i0 + q, j = j0 + tx;
        t[q][tx] = (i < n && j < n) ? H[(int64_t)(n - 1 - i) * ldh + (n - 1 - j)] : 0.0;
    }
    __syncthreads();
    for (int q = ty; q < 64; q += 4) {
        const int j = j0 + q, i = i0 + tx;
        if (i < n && j < n) Ht[(int64_t)j * ldh + i] = t[tx][q];
    }
}

// Off-diagonal row sums and diagonal of Ht: row i of Ht is column n-1-i of H.
__global__ __launch_bounds__(256) void ht_norms_kernel(int n, const double *H, int64_t ldh, double *offrow,
                                                       double *diag)
{
    const int i = blockIdx.x, c = n - 1 - i;
    const double *col = H + (int64_t)c * ldh;
    double acc = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) acc += r == c ? 0.0 : fabs(col[r]);
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        offrow[i] = red[0];
        diag[i] = col[c];
    }
}

// Build Ht and its norms on the first transposed solve (kept by the handle);
// every solve's stream then waits for them.
hipError_t ensure_transposed(shs_handle *h, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(h->ht_mu);
    if (!h->Ht) {
        const int64_t n = h->n;
        double *Ht = nullptr, *off = nullptr, *dg = nullptr;
        hipError_t e = hipMalloc((void **)&Ht, sizeof(double) * h->ldh * n);
        if (e == hipSuccess) e = hipMalloc((void **)&off, sizeof(double) * n);
        if (e == hipSuccess) e = hipMalloc((void **)&dg, sizeof(double) * n);
        if (e == hipSuccess && !h->ht_ready) e = hipEventCreateWithFlags(&h->ht_ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMemsetAsync(Ht, 0, sizeof(double) * h->ldh * n, st);   // padding rows
        if (e == hipSuccess) {
            hipLaunchKernelGGL(transpose_reverse_kernel, dim3(cdiv(n, 64), cdiv(n, 64)), dim3(256), 0, st, (int)n,
                               (const double *)h->H, h->ldh, Ht);
            hipLaunchKernelGGL(ht_norms_kernel, dim3((unsigned)n), dim3(256), 0, st, (int)n, (const double *)h->H,
                               h->ldh, off, dg);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(h->ht_ready, st);
        if (e != hipSuccess) {
            hipFree(Ht);
            hipFree(off);
            hipFree(dg);
            return e;
        }
        h->Ht = Ht;
        h->ht_offrow = off;
        h->ht_diag = dg;
        h->resident += sizeof(double) * (h->ldh * n + 2 * n);
        return hipSuccess;
    }
    return hipStreamWaitEvent(st, h->ht_ready, 0);
}

// Virtual items v = j nch + q (shift j, chunk q of m right-hand sides):
// their shifts, and E_v(i, c) = D(n-1-i, j r + q m + c) (zero past column r).
__global__ __launch_bounds__(256) void transposed_pack_kernel(int n, int m, int r, int nch, const double *shifts,
                                                              const double *D, int64_t ldd, double *shv, double *E)
{
    const int v = blockIdx.x, j = v / nch, q = v % nch;
    if (blockIdx.y == 0 && threadIdx.x < 2) shv[2 * v + threadIdx.x] = shifts[2 * j + threadIdx.x];
    const int64_t total = (int64_t)n * m;
    for (int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.y * 256) {
        const int c = (int)(idx / n), i = (int)(idx % n), k = q * m + c;
        double re = 0.0, im = 0.0;
        if (k < r) {
            const double *p = D + (((int64_t)j * r + k) * ldd + (n - 1 - i)) * 2;
            re = p[0];
            im = p[1];
        }
        double *e = E + (((int64_t)v * m + c) * n + i) * 2;
        e[0] = re;
        e[1] = im;
    }
}

// X(i, j r + k) = Xv(n-1-i, v m + c) with k = q m + c < r; per shift, eta is
// the largest of its items' and the status the first non-OK one.
__global__ __launch_bounds__(256) void transposed_unpack_kernel(int n, int m, int r, int nch, const double *Xv,
                                                                double *X, int64_t ldx, const double *etav,
                                                                const int32_t *stv, double *eta, int32_t *status)
{
    const int v = blockIdx.x, j = v / nch, q = v % nch;
    if (q == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        int st = 0;
        double e = 0.0;
        for (int qq = 0; qq < nch; ++qq) {
            const int s2 = stv[j * nch + qq];
            if (st == 0) st = s2;
            if (etav) {
                const double x = etav[j * nch + qq];
                e = (x > e || x != x) ? x : e;
            }
        }
        status[j] = st;
        if (eta && etav) eta[j] = e;
    }
    if (!X) return;
    const int cols = min(m, r - q * m);
    const int64_t total = (int64_t)n * cols;
    for (int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.y * 256) {
        const int c = (int)(idx / n), i = (int)(idx % n);
        const double *p = Xv + (((int64_t)v * m + c) * n + (n - 1 - i)) * 2;
        double *o = X + (((int64_t)j * r + q * m + c) * ldx + i) * 2;
        o[0] = p[0];
        o[1] = p[1];
    }
}

struct TransLayout {
    size_t shv = 0, e = 0, yd = 0, refl = 0, xv = 0, stv = 0, etav = 0, resmax = 0, xmax = 0, emax = 0, xt = 0;
    size_t zb = 0, bm = 0, m2 = 0, m2p = 0, m2q = 0;   // blocked sweep (m <= kBlkDenseMaxM)
    bool blocked = false;
    int64_t blk_rows = 0;
    size_t total = 0;
    int64_t nch = 0, nv = 0, refl_stride = 0;
};

bool trans_layout(const shs_handle *h, int64_t s, int64_t r, TransLayout *L)
{
    const int64_t n = h->n, m = h->m;
    Geo g;
    if (!geo(false, n, m, true, &g)) return false;
    L->nch = (r + m - 1) / m;
    L->nv = s * L->nch;
    L->refl_stride = g.stride;
    const int64_t nv = L->nv;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += al(bytes); return o; };
    L->shv = take(sizeof(double) * 2 * nv);
    L->e = take(sizeof(double) * 2 * n * m * nv);
    L->yd = take(sizeof(double) * 2 * n * m * nv);
    L->refl = take(sizeof(double) * g.stride * nv);
    L->xv = take(sizeof(double) * 2 * n * m * nv);
    L->stv = take(sizeof(int32_t) * nv);
    L->etav = take(sizeof(double) * nv);
    L->resmax = take(sizeof(unsigned long long) * m * nv);
    L->xmax = take(sizeof(unsigned long long) * m * nv);
    L->emax = take(sizeof(unsigned long long) * m * nv);
    L->xt = take(sizeof(double) * residual_pack_rows(n) * residual_pack_ld(m * nv));
    int tr = 0, w = 0;
    if (blk_geometry(false, (int)m, true, &tr, &w)) {
        // the blocked sweep with a dense right-hand side (Section 3.1, Step 2
        // revisited, with N_blk beside M_blk)
        L->blocked = true;
        const int64_t cols = blk_ncols(w, nv);
        L->blk_rows = (kBlkGroup * tr + m + 15) / 16 * 16;
        L->zb = take(sizeof(double) * n * cols);
        L->bm = take(sizeof(double) * L->blk_rows * cols);
        L->m2 = take(sizeof(double) * (cols / w) * w * w);
        L->m2p = take(sizeof(double) * (cols / w) * w * w);
        L->m2q = take(sizeof(double) * (cols / w) * w * w);
    }
    L->total = off;
    return true;
}

}  // namespace

namespace shs {

__global__ __launch_bounds__(256) void zero_fill_kernel(unsigned long long *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = 0ull;
}

hipError_t zero_fill(void *p, size_t bytes, hipStream_t st)
{
    const int64_t count = (int64_t)(bytes / 8);
    if (count <= 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(zero_fill_kernel, dim3(grid), dim3(256), 0, st, (unsigned long long *)p, count);
    return hipGetLastError();
}

// residual + eta for the listed shifts; Res optional.
hipError_t certify(shs_handle *h, int64_t s_list, const int32_t *dlist, const int *dcount, const double *shifts,
                   const double *X, int64_t ldx, double *Res, unsigned long long *resmax, unsigned long long *xmax,
                   double *eta, int32_t *status, int64_t s_total, double *Xt, hipStream_t st, const CertifyOpts *opt)
{
    const CertifyOpts none;
    if (!opt) opt = &none;
    const int64_t n = h->n, m = h->m;
    const int64_t nc = opt->nc > 0 ? opt->nc : m;
    const double *Hm = opt->H ? opt->H : h->H;
    // timed phases: the residual GEMM alone; clearing, packing and eta count
    // as other work
    PhaseScope ps0(h, PH_OTHER, s_list, st);
    hipError_t e = zero_fill(resmax, sizeof(unsigned long long) * nc * s_total, st);
    if (e != hipSuccess) return e;
    e = zero_fill(xmax, sizeof(unsigned long long) * nc * s_total, st);
    if (e != hipSuccess) return e;
    if (opt->E) {
        e = zero_fill(opt->emax, sizeof(unsigned long long) * nc * s_total, st);
        if (e != hipSuccess) return e;
    }
    ResidualArgs ra;
    ra.n = (int)n;
    ra.m = (int)m;
    ra.nc = (int)nc;
    ra.count = (int)s_list;
    ra.list = dlist;
    ra.H = Hm;
    ra.ldh = h->ldh;
    ra.Rtop = h->Rtop;
    ra.shifts = shifts;
    ra.X = X;
    ra.ldx = ldx;
    ra.Xt = Xt;
    ra.Res = Res;
    ra.ldr = n;
    ra.resmax = resmax;
    ra.xmax = xmax;
    ra.dcount = dcount;
    ra.E = opt->E;
    ra.lde = opt->lde;
    ra.emax = opt->emax;
    ra.ldxt = residual_pack_ld(s_list * nc);
    if (s_list <= 0) return hipGetLastError();
    // what the direct-to-LDS loads assume: 16-byte aligned pairs of rows
    if (n < 2 || h->ldh & 1 || ((uintptr_t)Hm | (uintptr_t)Xt) & 15) return hipErrorInvalidValue;
    if (!opt->E && nc != m) return hipErrorInvalidValue;
    hipLaunchKernelGGL(residual_pack_kernel, dim3(cdiv(residual_pack_rows(n), 64), ra.ldxt / 64), dim3(256), 0, st,
                       ra);
    ps0.end();
    {
        PhaseScope ps(h, PH_RESIDUAL, s_list, st);
        ra.ncol_tiles = (int)((cdiv(s_list * nc, 64) + 7) / 8 * 8);
        hipLaunchKernelGGL(residual_mfma_kernel, dim3((unsigned)(cdiv(n, 128) * ra.ncol_tiles)), dim3(256),
                           kResidualLds, st, ra);
    }
    PhaseScope ps1(h, PH_OTHER, s_list, st);
    hipLaunchKernelGGL(eta_kernel, dim3((unsigned)s_list), dim3(256), 0, st, (int)n, (int)nc, (int)s_list, dcount, dlist,
                       shifts, opt->offrow ? opt->offrow : (const double *)h->offrow,
                       opt->diag ? opt->diag : (const double *)h->diag, (const double *)h->rcolmax,
                       (const unsigned long long *)resmax, (const unsigned long long *)xmax,
                       (const unsigned long long *)opt->emax, eta, status);
    return hipGetLastError();
}

hipError_t dgemm(bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                 int64_t ldb, double *C, int64_t ldc, bool accumulate, double *part, size_t part_elems,
                 hipStream_t st)
{
    return gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, C, ldc, accumulate, part, part_elems, st);
}

hipError_t g_eval(shs_handle *h, int64_t s, const double *X, int64_t ldx, double *G, int64_t ldg, hipStream_t st)
{
    if (s <= 0 || h->p <= 0) return hipSuccess;
    hipLaunchKernelGGL(g_eval_kernel, dim3((unsigned)s), dim3(256), 0, st, (int)h->n, (int)h->p, (int)h->m,
                       (int)s, (const int32_t *)nullptr, (const double *)h->Ct, h->ldct, X, ldx, G, ldg);
    return hipGetLastError();
}



bool sweep_geometry(bool fp32, int m, bool dense, SweepGeometry *g)
{
    if (fp32)
        return sweep_geometry_f32_0(m, dense, g) || sweep_geometry_f32_1(m, dense, g) ||
               sweep_geometry_f32_2(m, dense, g) || sweep_geometry_f32_3(m, dense, g) ||
               sweep_geometry_f32_4(m, dense, g) || sweep_geometry_f32_5(m, dense, g);
    return sweep_geometry_f64_0(m, dense, g) || sweep_geometry_f64_1(m, dense, g) ||
           sweep_geometry_f64_2(m, dense, g) || sweep_geometry_f64_3(m, dense, g) ||
           sweep_geometry_f64_4(m, dense, g) || sweep_geometry_f64_5(m, dense, g);
}

bool launch_sweep(int m, bool dense, const SweepArgs<double> &a, hipStream_t st)
{
    return launch_sweep_f64_0(m, dense, a, st) || launch_sweep_f64_1(m, dense, a, st) ||
           launch_sweep_f64_2(m, dense, a, st) || launch_sweep_f64_3(m, dense, a, st) ||
           launch_sweep_f64_4(m, dense, a, st) || launch_sweep_f64_5(m, dense, a, st);
}

bool launch_sweep(int m, bool dense, const SweepArgs<float> &a, hipStream_t st)
{
    return launch_sweep_f32_0(m, dense, a, st) || launch_sweep_f32_1(m, dense, a, st) ||
           launch_sweep_f32_2(m, dense, a, st) || launch_sweep_f32_3(m, dense, a, st) ||
           launch_sweep_f32_4(m, dense, a, st) || launch_sweep_f32_5(m, dense, a, st);
}

bool launch_qstar(int m, bool dense_in, const QstarArgs<double> &a, hipStream_t st)
{
    return launch_qstar_f64_0(m, dense_in, a, st) || launch_qstar_f64_1(m, dense_in, a, st) ||
           launch_qstar_f64_2(m, dense_in, a, st) || launch_qstar_f64_3(m, dense_in, a, st) ||
           launch_qstar_f64_4(m, dense_in, a, st) || launch_qstar_f64_5(m, dense_in, a, st);
}

bool launch_qstar(int m, bool dense_in, const QstarArgs<float> &a, hipStream_t st)
{
    return launch_qstar_f32_0(m, dense_in, a, st) || launch_qstar_f32_1(m, dense_in, a, st) ||
           launch_qstar_f32_2(m, dense_in, a, st) || launch_qstar_f32_3(m, dense_in, a, st) ||
           launch_qstar_f32_4(m, dense_in, a, st) || launch_qstar_f32_5(m, dense_in, a, st);
}

}  // namespace shs

namespace {

constexpr size_t kReducePart = (size_t)1 << 22;   // split-K workspace of the reduction's GEMMs (32 MiB)

// Blocked m-Hessenberg reduction of h->H (after the similarity with Q_B),
// following Algorithms 2 and 3: panels of b columns, mini-blocks of m.
//   For a panel starting at column z (reflectors on rows >= r_lo = z + m):
//   per mini-block q0 .. q0+mb-1 (columns j0 = z + q0 ..):
//     1. right update by the panel's earlier mini-blocks: A(:, mb cols) -= Y V(mb rows, :)^T
//     2. left update by the panel's earlier reflectors:  A(r_lo:, mb cols) -= V T^T V^T A(r_lo:, mb cols)
//     3. the mini-block's own reflectors (miniblock_kernel), its T block
//     4. T12 = -T_old (V_old^T V_new) T_new
//     5. Y_new = (A(:, j0+m:) V_new - Y_old (V_old^T V_new)) T_new
//   then the trailing columns c >= z + b: right A -= Y V^T, left A -= V T^T V^T A,
//   and C <- C (I - V T V^T).  Y = A V T always refers to the panel-start A;
//   the columns it reads (>= j0 + m) are still untouched when it is formed.
hipError_t reduce_blocked(shs_handle *h, double *work, hipStream_t st, LaunchCheck *chk = nullptr)
{
    const int n = (int)h->n, m = (int)h->m, p = (int)h->p;
    const int b = std::max(m, (64 / m) * m);
    double *H = h->H;
    const int64_t ldh = h->ldh;
    double *Vp = work;                        // n x b
    double *Y = Vp + (size_t)n * b;           // n x b
    double *Z = Y + (size_t)n * b;            // n x m
    double *Tp = Z + (size_t)n * m;           // b x b
    double *S = Tp + (size_t)b * b;           // b x m
    double *U = S + (size_t)b * m;            // b x m
    double *W = U + (size_t)b * m;            // b x n
    double *W2 = W + (size_t)b * n;           // b x n
    double *CV = W2 + (size_t)b * n;          // max(1,p) x b
    double *CVT = CV + (size_t)std::max(1, p) * b;
    double *taus = CVT + (size_t)std::max(1, p) * b;   // b
    double *part = taus + b;                            // split-K partials
    const int ldp = std::max(1, p);
    hipError_t e = hipSuccess;
#define GEMM(...)                                         \
    do {                                                  \
        e = gemm_f64(__VA_ARGS__, part, kReducePart, st, chk); \
        if (e != hipSuccess) return e;                    \
    } while (0)
    const int nref = n - m - 1;   // columns that get a reflector
    for (int z = 0; z < nref; z += b) {
        const int bz = std::min(b, nref - z);
        const int r_lo = z + m, L = n - r_lo;
        // rows above each vector's first row are read by the GEMMs as zeros
        if (!chk) {
            e = hipMemsetAsync(Vp, 0, sizeof(double) * n * b, st);
            if (e != hipSuccess) return e;
            e = hipMemsetAsync(Tp, 0, sizeof(double) * b * b, st);
            if (e != hipSuccess) return e;
        }
        for (int q0 = 0; q0 < bz; q0 += m) {
            const int mb = std::min(m, bz - q0);
            const int j0 = z + q0;
            double *Acols = H + (int64_t)j0 * ldh;
            if (q0 > 0) {
                // 1. right update by earlier mini-blocks (all rows)
                GEMM(false, true, n, mb, q0, -1.0, Y, n, Vp + j0, n, Acols, ldh, true);
                // 2. left update by earlier reflectors (rows r_lo ..)
                GEMM(true, false, q0, mb, L, 1.0, Vp + r_lo, n, Acols + r_lo, ldh, S, b, false);
                GEMM(true, false, q0, mb, q0, 1.0, Tp, b, S, b, U, b, false);
                GEMM(false, false, L, mb, q0, -1.0, Vp + r_lo, n, U, b, Acols + r_lo, ldh, true);
            }
            // 3. this mini-block's reflectors and T block
            if (!chk) {
                hipLaunchKernelGGL(miniblock_kernel, dim3(1), dim3(1024), 0, st, n, m, r_lo, j0, mb, q0, H, ldh, Vp,
                                   taus, Tp, b);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            const double *Vnew = Vp + (int64_t)q0 * n;
            if (q0 > 0) {
                // 4. S = V_old^T V_new; T12 = -T_old S T_new
                GEMM(true, false, q0, mb, L, 1.0, Vp + r_lo, n, Vnew + r_lo, n, S, b, false);
                GEMM(false, false, q0, mb, mb, 1.0, S, b, Tp + (int64_t)q0 * b + q0, b, U, b, false);
                GEMM(false, false, q0, mb, q0, -1.0, Tp, b, U, b, Tp + (int64_t)q0 * b, b, false);
            }
            // 5. Y_new = (A(:, j0+m:) V_new - Y_old S) T_new
            const int c1 = j0 + m;
            GEMM(false, false, n, mb, n - c1, 1.0, H + (int64_t)c1 * ldh, ldh, Vnew + c1, n, Z, n, false);
            if (q0 > 0) GEMM(false, false, n, mb, q0, -1.0, Y, n, S, b, Z, n, true);
            GEMM(false, false, n, mb, mb, 1.0, Z, n, Tp + (int64_t)q0 * b + q0, b, Y + (int64_t)q0 * n, n, false);
        }
        // trailing columns
        const int c0 = z + bz, N = n - c0;
        if (N > 0) {
            double *At = H + (int64_t)c0 * ldh;
            GEMM(false, true, n, N, bz, -1.0, Y, n, Vp + c0, n, At, ldh, true);
            GEMM(true, false, bz, N, L, 1.0, Vp + r_lo, n, At + r_lo, ldh, W, b, false);
            GEMM(true, false, bz, N, bz, 1.0, Tp, b, W, b, W2, b, false);
            GEMM(false, false, L, N, bz, -1.0, Vp + r_lo, n, W2, b, At + r_lo, ldh, true);
        }
        if (p > 0) {
            GEMM(false, false, p, bz, L, 1.0, h->Ct + (int64_t)r_lo * h->ldct, h->ldct, Vp + r_lo, n, CV, ldp, false);
            GEMM(false, false, p, bz, bz, 1.0, CV, ldp, Tp, b, CVT, ldp, false);
            GEMM(false, true, p, L, bz, -1.0, CVT, ldp, Vp + r_lo, n, h->Ct + (int64_t)r_lo * h->ldct, h->ldct, true);
        }
        // keep the reflectors for Q (apply_q): reflector m + z + q
        if (chk) {
            if (!chk->inside(h->V + (int64_t)(m + z) * n, (int64_t)n * bz - 1) ||
                !chk->inside(h->tauv + m + z, bz - 1))
                chk->fail("reflector copy", n, bz, 0);
            continue;
        }
        e = hipMemcpyAsync(h->V + (int64_t)(m + z) * n, Vp, sizeof(double) * n * bz, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(h->tauv + m + z, taus, sizeof(double) * bz, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
#undef GEMM
    return chk ? hipSuccess : hipGetLastError();
}

// Mixed precision (complex FP32 sweep + FP64 iterative refinement), all on
// the stream: the shifts still being refined, and those that fall back to
// the FP64 sweep, are kept in device lists whose lengths the kernels read on
// the device, so the host never waits.  Every round launches its kernels for
// up to s shifts; launches past a list's length exit at once.
//   X = Q* (FP32 sweep of all shifts)
//   for it = 0 .. max_iter:
//       eta of the listed shifts (FP64 residual GEMM); split the list into
//       done / next / fallback (mixed_select_kernel); stop at it = max_iter
//       correction of the next list: (H - sigma I) D = Res / scale in FP32
//       (dense right-hand side), X += scale D
//   FP64 (blocked) sweep and eta of the fallback list; their status.
hipError_t solve_mixed(shs_handle *h, int64_t s, const double *shifts, double tol, int max_iter, void *work,
                       const Layout &L, double *Xw, int64_t ldxw, double *eta, int32_t *status, hipStream_t st)
{
    const int64_t n = h->n, m = h->m;
    Geo g32s, g32d;
    geo(true, n, m, false, &g32s);
    geo(true, n, m, true, &g32d);
    int32_t *lists[2] = {at<int32_t>(work, L.list), at<int32_t>(work, L.list2)};
    int32_t *fbl = at<int32_t>(work, L.fblist);
    int *cnt = at<int>(work, L.cnt);
    int32_t *st2 = at<int32_t>(work, L.status2);
    double *Res = at<double>(work, L.res);
    long long *stats = h->timing ? h->dstats : nullptr;
    hipError_t e = hipSuccess;
    {
        PhaseScope ps(h, PH_OTHER, s, st);
        hipLaunchKernelGGL(mixed_init_kernel, dim3(cdiv(s, 256)), dim3(256), 0, st, (int)s, lists[0],
                           at<double>(work, L.eta_prev), cnt, stats);
    }
    SweepArgs<float> sa{};
    sa.n = (int)n;
    sa.count = (int)s;
    sa.H = h->H32;
    sa.ldh = h->ldh;
    sa.shifts = shifts;
    sa.list = nullptr;
    sa.Rtop = h->Rtop;
    sa.refl = at<float>(work, L.refl32);
    sa.refl_stride = L.refl32_stride;
    sa.Y = at<float>(work, L.y32);
    sa.y_stride = 2 * m * m;
    sa.status = st2;
    // the FP32 sweeps run blocked (Section 3.1, Step 2 revisited) on the FP32
    // matrix cores; their reflector stores follow the blocked tile height
    const BlkBufT<float> B32{at<float>(work, L.z32), at<float>(work, L.bm32), at<float>(work, L.m2a),
                             at<float>(work, L.m2b), at<float>(work, L.m2c), L.blk32_rows};
    int trs = 0, ws = 0, trd = 0, wd = 0;
    blk_geometry(true, (int)m, false, &trs, &ws);
    blk_geometry(true, (int)m, true, &trd, &wd);
    e = sweep_blocked<float>(h, s, nullptr, nullptr, shifts, B32, sa, st, nullptr, h->H32, PH_SWEEP32);
    if (e != hipSuccess) return e;
    QstarArgs<float> qa{};
    qa.n = (int)n;
    qa.count = (int)s;
    qa.list = nullptr;
    qa.refl = sa.refl;
    qa.refl_stride = L.refl32_stride;
    qa.tile_rows = trs;
    qa.tile_stride = refl_tile_stride<float>(trs, slot_elems((int)m, false));
    qa.slot = slot_elems((int)m, false);
    qa.Y = sa.Y;
    qa.y_stride = 2 * m * m;
    qa.X = Xw;
    qa.ldx = ldxw;
    qa.accumulate = 0;
    {
        PhaseScope ps(h, PH_QSTAR, s, st);
        if (!launch_qstar((int)m, false, qa, st)) return hipErrorInvalidValue;
    }
    for (int it = 0;; ++it) {
        int32_t *in = lists[it & 1], *out = lists[(it + 1) & 1];
        const int *cin = cnt + (it & 1);
        int *cout = cnt + ((it + 1) & 1);
        e = certify(h, s, in, cin, shifts, Xw, ldxw, Res, at<unsigned long long>(work, L.resmax),
                    at<unsigned long long>(work, L.xmax), eta, nullptr, s, at<double>(work, L.xt), st);
        if (e != hipSuccess) return e;
        {
            PhaseScope ps(h, PH_OTHER, s, st);
            hipLaunchKernelGGL(mixed_select_kernel, dim3(1), dim3(1024), 0, st, it, max_iter, tol,
                               (const int32_t *)in, cin, out, cout, fbl, cnt + 2, (const double *)eta,
                               at<double>(work, L.eta_prev), status, stats);
        }
        if (it >= max_iter) break;
        // correction: (H - sigma I) D = Res in FP32 (scaled), X += scale D
        {
            PhaseScope ps(h, PH_OTHER, s, st);
            hipLaunchKernelGGL(scale_residual_kernel, dim3((unsigned)s, std::max<unsigned>(1, cdiv(n * m, 256 * 16))),
                               dim3(256), 0, st, (int)n, (int)m, (const int *)cout, (const int32_t *)out,
                               (const double *)Res, (const unsigned long long *)at<unsigned long long>(work, L.resmax),
                               at<double>(work, L.scale), at<float>(work, L.e32));
        }
        SweepArgs<float> da{};
        da.n = (int)n;
        da.count = (int)s;
        da.H = h->H32;
        da.ldh = h->ldh;
        da.shifts = shifts;
        da.list = out;
        da.Rtop = h->Rtop;
        da.E = at<float>(work, L.e32);
        da.e_stride = 2 * n * m;
        da.refl = at<float>(work, L.refl32);
        da.refl_stride = L.refl32_stride;
        da.Y = at<float>(work, L.yd32);
        da.y_stride = 2 * n * m;
        da.status = st2;
        da.dcount = cout;
        QstarArgs<float> dq{};
        if (L.blk32_dense) {
            // blocked, N_blk beside M_blk
            e = sweep_blocked<float>(h, s, out, cout, shifts, B32, da, st, at<float>(work, L.e32), h->H32,
                                     PH_SWEEP32D);
            if (e != hipSuccess) return e;
            dq.tile_rows = trd;
            dq.tile_stride = refl_tile_stride<float>(trd, slot_elems((int)m, true));
        } else {
            PhaseScope ps(h, PH_SWEEP32D, s, st);
            if (!launch_sweep((int)m, true, da, st)) return hipErrorInvalidValue;
            dq.tile_rows = g32d.g.tile_rows;
            dq.tile_stride = g32d.g.tile_stride;
        }
        dq.n = (int)n;
        dq.count = (int)s;
        dq.list = out;
        dq.refl = da.refl;
        dq.refl_stride = L.refl32_stride;
        dq.slot = g32d.g.slot;
        dq.Y = da.Y;
        dq.y_stride = 2 * n * m;
        dq.X = Xw;
        dq.ldx = ldxw;
        dq.accumulate = 1;
        dq.scale = at<double>(work, L.scale);
        dq.dcount = cout;
        {
            PhaseScope ps(h, PH_QSTAR, s, st);
            if (!launch_qstar((int)m, true, dq, st)) return hipErrorInvalidValue;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // FP64 sweep for the shifts the mixed form could not certify (the
    // refinement buffers are dead now; the blocked sweep reuses them)
    e = solve_fp64(h, s, fbl, cnt + 2, shifts, work, L, Xw, ldxw, st2, st);
    if (e != hipSuccess) return e;
    e = certify(h, s, fbl, cnt + 2, shifts, Xw, ldxw, nullptr, at<unsigned long long>(work, L.resmax),
                at<unsigned long long>(work, L.xmax), eta, st2, s, at<double>(work, L.xt), st);
    if (e != hipSuccess) return e;
    {
        PhaseScope ps(h, PH_OTHER, s, st);
        hipLaunchKernelGGL(mixed_final_kernel, dim3(cdiv(s, 256)), dim3(256), 0, st, (const int *)(cnt + 2),
                           (const int32_t *)fbl, (const int32_t *)st2, (const double *)eta, tol, status);
    }
    return hipGetLastError();
}

size_t reduce_blocked_work(int64_t n, int64_t m, int64_t p)
{
    const int64_t b = std::max(m, (64 / m) * m);
    return sizeof(double) * ((size_t)(2 * n * b + n * m + b * b + 2 * b * m + 2 * b * n +
                                      2 * std::max<int64_t>(1, p) * b + b) +
                             kReducePart);
}

// ---- per-shift directions (Section 3.3) -----------------------------------
// The interpolation method solves (A - sigma_j I) x_j = B b_j and
// (A - sigma_j I)^T w_j = C^T c_j with directions b_j (m) and c_j (p) of
// their own per shift.  In reduced coordinates the first right-hand side is
// R b_j, nonzero in its first m rows only, so the structured sweep applies
// unchanged and only its end differs: y_j = R_sigma(0:m,0:m)^{-1} R(0:m,0:m) b_j
// and x_j = Q_sigma^*(:, 0:m) y_j.  The second one, Ct^T c_j, is dense and
// goes through the transposed solve.

// X(:, j) = Xm(:, j m) (the only nonzero column of the shift's Q* output) and,
// for the backward error, E(:, j) = [R(0:m,0:m) b_j; 0].
__global__ __launch_bounds__(256) void vec_out_kernel(int n, int m, const double *Xm, double *X, int64_t ldx,
                                                      const double *Rtop, const double *bhat, int64_t ldb, double *E)
{
    const int j = blockIdx.x;
    const double *src = Xm + (int64_t)j * m * n * 2;
    const double *b = bhat + (int64_t)j * ldb * 2;
    for (int i = blockIdx.y * 256 + threadIdx.x; i < n; i += gridDim.y * 256) {
        if (X) {
            X[((int64_t)j * ldx + i) * 2] = src[2 * i];
            X[((int64_t)j * ldx + i) * 2 + 1] = src[2 * i + 1];
        }
        if (E) {
            double er = 0.0, ei = 0.0;
            for (int c = i; c < m; ++c) {   // R(0:m,0:m) is upper triangular
                er = fma(Rtop[c * m + i], b[2 * c], er);
                ei = fma(Rtop[c * m + i], b[2 * c + 1], ei);
            }
            E[((int64_t)j * n + i) * 2] = er;
            E[((int64_t)j * n + i) * 2 + 1] = ei;
        }
    }
}

// Transposed systems with directions: E_j(i, 0) = (Ct^T c_j)(n-1-i) (the
// order-reversed right-hand side of the sweep of J H^T J), E_j(i, c) = 0 for
// c >= 1; D_j(i) = (Ct^T c_j)(i) when D is set (for the backward error).
__global__ __launch_bounds__(256) void tvec_pack_kernel(int n, int m, int p, const double *Ct, int64_t ldct,
                                                        const double *chat, int64_t ldc, double *E)
{
    const int j = blockIdx.x;
    const double *c = chat + (int64_t)j * ldc * 2;
    const int64_t total = (int64_t)n * m;
    for (int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.y * 256) {
        const int col = (int)(idx / n), i = (int)(idx % n);
        double er = 0.0, ei = 0.0;
        if (col == 0) {
            const int r = n - 1 - i;
            for (int q = 0; q < p; ++q) {
                const double w = Ct[(int64_t)r * ldct + q];
                er = fma(w, c[2 * q], er);
                ei = fma(w, c[2 * q + 1], ei);
            }
        }
        double *e = E + (((int64_t)j * m + col) * n + i) * 2;
        e[0] = er;
        e[1] = ei;
    }
}

// ---- X <- Q X in blocks of reflectors ------------------------------------
constexpr int64_t kApplyQBlock = 64;

// Xr(:, c) = Re X(:, c), Xr(:, ncols + c) = Im X(:, c) (Xr: n x 2 ncols, ld n)
__global__ __launch_bounds__(256) void split_complex_kernel(int n, const double *X, int64_t ld, double *Xr, int ncols)
{
    const int i = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
    if (i >= n) return;
    const double *x = X + ((int64_t)c * ld + i) * 2;
    Xr[(int64_t)c * n + i] = x[0];
    Xr[(int64_t)(ncols + c) * n + i] = x[1];
}

__global__ __launch_bounds__(256) void join_complex_kernel(int n, const double *Xr, int ncols, double *X, int64_t ld)
{
    const int i = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
    if (i >= n) return;
    double *x = X + ((int64_t)c * ld + i) * 2;
    x[0] = Xr[(int64_t)c * n + i];
    x[1] = Xr[(int64_t)(ncols + c) * n + i];
}

// T of the compact WY form H_0 H_1 ... H_{b-1} = I - V T V^T (T upper
// triangular, b x b, ld ldt = blockDim.x) from G = V^T V and the taus:
// T(i, i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i).  One workgroup,
// thread k owns row k.
__global__ __launch_bounds__(64) void wy_t_kernel(int b, const double *G, int ldg, const double *tau, double *T)
{
    const int k = threadIdx.x, ldt = blockDim.x;
    for (int e = k; e < ldt * ldt; e += blockDim.x) T[e] = 0.0;
    __syncthreads();
    for (int i = 0; i < b; ++i) {
        const double ti = tau[i];
        double s = 0.0;
        if (k < i)
            for (int l = k; l < i; ++l) s = fma(T[(int64_t)l * ldt + k], G[(int64_t)i * ldg + l], s);
        __syncthreads();
        if (k < i) T[(int64_t)i * ldt + k] = -ti * s;
        if (k == i) T[(int64_t)i * ldt + i] = ti;
        __syncthreads();
    }
}

// Workspace of shs_solve_vec: the FP64 solve's layout with a Q* output of m
// columns per shift, then the right-hand sides [R b_j; 0] and their maxima.
struct VecLayout {
    Layout base;
    size_t e = 0, emax = 0, total = 0;
};

bool vec_layout(const shs_handle *h, int64_t s, VecLayout *V)
{
    if (!layout(h, s, SHS_MODE_FP64, SHS_OUT_G, &V->base)) return false;   // no X output: Q* into the workspace
    size_t off = V->base.total;
    auto take = [&](size_t bytes) { size_t o = off; off += al(bytes); return o; };
    V->e = take(sizeof(double) * 2 * h->n * s);
    V->emax = take(sizeof(unsigned long long) * s);
    V->total = off;
    return true;
}

}  // namespace

// ---- scratch of shs_solve_noalloc ------------------------------------------
// One array per GPU the library runs on (the code object holds it; the GPU
// keeps it until the process ends).  Host code must not use the name
// `scratch` as an address: it is a host-side stand-in.  Its device address
// is taken once per device with hipGetSymbolAddress and kept in
// g_scratch_ptr, which is what kernels and copies receive.
constexpr size_t kNoAllocBytes = SHS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current.
hipError_t noalloc_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidValue;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

#define RETURN_IF_HIP(expr)                                        \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) {                                    \
            if (e_ == hipErrorOutOfMemory) return SHS_ERR_NOMEM;   \
            return SHS_ERR_HIP;                                    \
        }                                                          \
    } while (0)

extern "C" {

int shs_abi_version(void) { return SHS_ABI_VERSION; }

const char *shs_strerror(int code)
{
    if (code < 0) return "invalid argument";
    switch (code) {
    case 0: return "success";
    case SHS_ERR_NOMEM: return "out of device memory or over budget";
    case SHS_ERR_HIP: return "HIP runtime error";
    case SHS_ERR_UNSUPPORTED: return "unsupported shape";
    case SHS_ERR_BUSY: return "busy";
    case SHS_ERR_NOTFOUND: return "unknown id";
    case SHS_ERR_TIMEOUT: return "timed out";
    case SHS_ERR_CANCELLED: return "cancelled";
    case SHS_ERR_STATE: return "request already finished or not finished";
    case SHS_ERR_SCRATCH: return "the solve needs more than the static scratch of shs_solve_noalloc";
    default: return "unknown error";
    }
}

int shs_reduce(int64_t n, int64_t m, int64_t p, const double *A, int64_t lda, const double *B, int64_t ldb,
               const double *C, int64_t ldc, const shs_config *cfg, void *stream, shs_handle **out)
{
    if (n < 2) return -1;
    if (m < 1 || m >= n) return -2;
    if (m > SHS_MAX_M) return SHS_ERR_UNSUPPORTED;
    if (p < 0) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!B) return -6;
    if (ldb < n) return -7;
    if (p > 0 && !C) return -8;
    if (ldc < std::max<int64_t>(1, p)) return -9;
    if (cfg && cfg->abi_version != SHS_ABI_VERSION) return -10;
    if (!out) return -12;
    if (n > (int64_t)INT32_MAX / 2) return SHS_ERR_UNSUPPORTED;
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;

    shs_handle *h = new (std::nothrow) shs_handle();
    if (!h) return SHS_ERR_NOMEM;
    h->n = n;
    h->m = m;
    h->p = p;
    hipGetDevice(&h->device);
    h->ldh = (n + 15) / 16 * 16;   // 16-byte aligned pairs of rows in every column
    h->ldct = std::max<int64_t>(1, p);
    h->nrefl = m + std::max<int64_t>(0, n - m - 1);
    size_t acc = 0;
    hipError_t e = hipSuccess;
    double *part = nullptr, *bwork = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
#define ALLOC(ptr, cnt)                                \
    do {                                               \
        e = dmalloc(&(ptr), (size_t)(cnt), &acc);      \
        if (e != hipSuccess) goto fail;                \
    } while (0)
    ALLOC(h->H, h->ldh * n);
    ALLOC(h->H32, h->ldh * n);
    ALLOC(h->Bw, n * m);
    ALLOC(h->Rtop, m * m);
    ALLOC(h->rcolmax, m);
    ALLOC(h->Ct, h->ldct * n);
    ALLOC(h->V, n * h->nrefl);
    ALLOC(h->tauv, h->nrefl);
    ALLOC(h->sgn, n);
    ALLOC(h->offrow, n);
    ALLOC(h->diag, n);
    ALLOC(h->dstats, 4);
#undef ALLOC
    e = hipMalloc((void **)&part, sizeof(double) * (size_t)std::max<int64_t>(n, 1) * cdiv(n, kRightChunk));
    if (e != hipSuccess) goto fail;
    e = hipMalloc((void **)&bwork, reduce_blocked_work(n, m, p));
    if (e != hipSuccess) goto fail;
    h->resident = acc;

    e = hipEventCreate(&e0);
    if (e != hipSuccess) goto fail;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) goto fail;
    e = hipEventRecord(e0, st);
    if (e != hipSuccess) goto fail;

    e = hipMemsetAsync(h->H, 0, sizeof(double) * h->ldh * n, st);   // padding rows stay zero
    if (e != hipSuccess) goto fail;
    e = hipMemcpy2DAsync(h->H, sizeof(double) * h->ldh, A, sizeof(double) * lda, sizeof(double) * n, n,
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) goto fail;
    e = hipMemcpy2DAsync(h->Bw, sizeof(double) * n, B, sizeof(double) * ldb, sizeof(double) * n, m,
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) goto fail;
    if (p > 0) {
        e = hipMemcpy2DAsync(h->Ct, sizeof(double) * h->ldct, C, sizeof(double) * ldc, sizeof(double) * p, n,
                             hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) goto fail;
    }
    e = hipMemsetAsync(h->V, 0, sizeof(double) * n * h->nrefl, st);
    if (e != hipSuccess) goto fail;

    // 1.-2. QR of B and the similarity with Q_B
    for (int64_t j = 0; j < m; ++j) {
        const int64_t L = n - j;
        double *v = h->V + j * n + j;
        double *tau = h->tauv + j;
        hipLaunchKernelGGL(house_kernel, dim3(1), dim3(1024), 0, st, (int)L, h->Bw + j * n + j, v, tau);
        if (m - j - 1 > 0)
            hipLaunchKernelGGL(left_update_kernel, dim3((unsigned)(m - j - 1)), dim3(256), 0, st, (int)L, (int)j,
                               (int)(j + 1), h->Bw, (int64_t)n, (const double *)v, (const double *)tau);
        e = two_sided(h, h->H, h->ldh, L, j, 0, v, tau, part, st);
        if (e != hipSuccess) goto fail;
    }
    // 3.-4. m-Hessenberg reduction, blocked (reflector j annihilates H(j+m+1:, j))
    e = reduce_blocked(h, bwork, st);
    if (e != hipSuccess) goto fail;
    // sign normalisation and derived data
    hipLaunchKernelGGL(signs_kernel, dim3(1), dim3(64), 0, st, (int)n, (int)m, (const double *)h->H, h->ldh,
                       (const double *)h->Bw, (int64_t)n, h->sgn);
    hipLaunchKernelGGL(finalize_h_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, (int)n, (int)m, h->H, h->ldh,
                       h->H32, (const double *)h->sgn, h->offrow, h->diag);
    hipLaunchKernelGGL(finalize_r_kernel, dim3(1), dim3(64), 0, st, (int)n, (int)m, h->Bw, (int64_t)n,
                       (const double *)h->sgn, h->Rtop, h->rcolmax);
    if (p > 0)
        hipLaunchKernelGGL(scale_cols_kernel, dim3(cdiv(p * n, 256)), dim3(256), 0, st, (int)p, (int)n, h->Ct,
                           h->ldct, (const double *)h->sgn);
    e = hipGetLastError();
    if (e != hipSuccess) goto fail;
    e = hipEventRecord(e1, st);
    if (e != hipSuccess) goto fail;
    e = hipEventSynchronize(e1);
    if (e != hipSuccess) goto fail;
    {
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        h->reduce_ms = ms;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(part);
    hipFree(bwork);
    *out = h;
    return 0;
fail:
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(part);
    hipFree(bwork);
    free_handle(h);
    return e == hipErrorOutOfMemory ? SHS_ERR_NOMEM : SHS_ERR_HIP;
}

int shs_reduce_check_plan(int64_t n, int64_t m, int64_t p, int64_t *launches, char *msg, int64_t msg_len)
{
    if (n < 2) return -1;
    if (m < 1 || m >= n || m > SHS_MAX_M) return -2;
    if (p < 0) return -3;
    if (n > (int64_t)INT32_MAX / 2) return SHS_ERR_UNSUPPORTED;
    // the allocations shs_reduce makes, at distinct addresses that are never
    // dereferenced (1 TiB apart, 256-byte aligned like hipMalloc's)
    shs_handle h;
    h.n = n;
    h.m = m;
    h.p = p;
    h.ldh = (n + 15) / 16 * 16;
    h.ldct = std::max<int64_t>(1, p);
    h.nrefl = m + std::max<int64_t>(0, n - m - 1);
    LaunchCheck chk;
    uintptr_t base = (uintptr_t)1 << 40;
    auto region = [&](size_t elems, const char *name) {
        double *p0 = reinterpret_cast<double *>(base);
        chk.add(p0, std::max<size_t>(elems, 1), name);
        base += (uintptr_t)1 << 40;
        return p0;
    };
    h.H = region((size_t)(h.ldh * n), "H");
    h.Ct = region((size_t)(h.ldct * n), "Ct");
    h.V = region((size_t)(n * h.nrefl), "V");
    h.tauv = region((size_t)h.nrefl, "tau");
    double *bwork = region(reduce_blocked_work(n, m, p) / sizeof(double), "work");
    hipError_t e = reduce_blocked(&h, bwork, nullptr, &chk);
    h.H = nullptr;   // the handle owns nothing here
    h.Ct = h.V = h.tauv = nullptr;
    if (launches) *launches = chk.launches;
    if (msg && msg_len > 0) snprintf(msg, (size_t)msg_len, "%s", chk.violations ? chk.first : "");
    if (e != hipSuccess) return SHS_ERR_HIP;
    return (int)std::min<int64_t>(chk.violations, INT32_MAX);
}

int shs_solve_workspace(const shs_handle *h, int64_t s, int mode, int outputs, size_t *bytes)
{
    if (!h) return -1;
    if (s < 0) return -2;
    if (mode != SHS_MODE_FP64 && mode != SHS_MODE_FP32_REFINE) return -3;
    if (!(outputs & (SHS_OUT_X | SHS_OUT_G))) return -4;
    if (!bytes) return -5;
    Layout L;
    if (!layout(h, s, mode, outputs, &L)) return SHS_ERR_UNSUPPORTED;
    *bytes = L.total;
    return 0;
}

int shs_solve_noalloc(shs_handle *h, int64_t s, const double *shifts, int mode, int outputs, double tol,
                      int max_iter, double *X, int64_t ldx, double *G, int64_t ldg, double *eta, int32_t *status,
                      void *stream)
{
    if (!h) return -1;
    if (s < 0 || s > INT32_MAX / 64) return -2;
    if (mode != SHS_MODE_FP64 && mode != SHS_MODE_FP32_REFINE) return -4;
    if (!(outputs & (SHS_OUT_X | SHS_OUT_G))) return -5;
    if (s == 0) return 0;
    if (h->timing) return SHS_ERR_STATE;   // phase timing creates events and grows host vectors
    Layout L;
    if (!layout(h, s, mode, outputs, &L)) return SHS_ERR_UNSUPPORTED;
    if (L.total > kNoAllocBytes) return SHS_ERR_SCRATCH;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SHS_ERR_HIP;
    if (dev != h->device) return SHS_ERR_STATE;
    void *ptr = nullptr;
    const hipError_t e = noalloc_scratch(dev, &ptr);
    if (e != hipSuccess) return SHS_ERR_HIP;
    // every buffer the solve reads before writing it is cleared by its own
    // kernels (the same holds for a fresh allocation), so what the previous
    // call left in the array does not matter
    return shs_solve(h, s, shifts, mode, outputs, tol, max_iter, ptr, kNoAllocBytes, X, ldx, G, ldg, eta, status,
                     stream);
}

int shs_solve(shs_handle *h, int64_t s, const double *shifts, int mode, int outputs, double tol, int max_iter,
              void *work, size_t work_bytes, double *X, int64_t ldx, double *G, int64_t ldg, double *eta,
              int32_t *status, void *stream)
{
    if (!h) return -1;
    if (s < 0 || s > INT32_MAX / 64) return -2;
    if (s > 0 && !shifts) return -3;
    if (mode != SHS_MODE_FP64 && mode != SHS_MODE_FP32_REFINE) return -4;
    if (!(outputs & (SHS_OUT_X | SHS_OUT_G))) return -5;
    if (mode == SHS_MODE_FP32_REFINE && !(tol > 0.0)) return -6;
    if (max_iter < 0) return -7;
    if (s == 0) return 0;   // nothing to do; the output pointers are not referenced
    if ((outputs & SHS_OUT_X) && (!X || ldx < h->n)) return -10;
    if ((outputs & SHS_OUT_G) && h->p > 0 && (!G || ldg < h->p)) return -12;
    if (((outputs & SHS_OUT_ETA) || mode == SHS_MODE_FP32_REFINE) && !eta) return -14;
    if (!status) return -15;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n, m = h->m;
    Layout L;
    if (!layout(h, s, mode, outputs, &L)) return SHS_ERR_UNSUPPORTED;
    if (h->timing) {   // timing state is only touched when enabled (see shs_set_timing)
        h->marks.clear();
        h->last_mixed = mode == SHS_MODE_FP32_REFINE;
        h->tile_flops = h->update_flops = 0.0;
    }
    bool owned = false;
    if (work) {
        if (work_bytes < L.total) return -9;
    } else {
        RETURN_IF_HIP(hipMallocAsync(&work, L.total, st));
        owned = true;
    }
    double *Xw = (outputs & SHS_OUT_X) ? X : at<double>(work, L.x);
    const int64_t ldxw = (outputs & SHS_OUT_X) ? ldx : n;
    int rc = 0;
    hipError_t e = hipSuccess;

    if (mode == SHS_MODE_FP64) {
        e = solve_fp64(h, s, nullptr, nullptr, shifts, work, L, Xw, ldxw, status, st);
        if (e == hipSuccess && (outputs & SHS_OUT_ETA))
            e = certify(h, s, nullptr, nullptr, shifts, Xw, ldxw, nullptr, at<unsigned long long>(work, L.resmax),
                        at<unsigned long long>(work, L.xmax), eta, status, s, at<double>(work, L.xt), st);
    } else {
        e = solve_mixed(h, s, shifts, tol, max_iter, work, L, Xw, ldxw, eta, status, st);
    }
    if (e == hipSuccess && (outputs & SHS_OUT_G) && h->p > 0) {
        PhaseScope ps(h, PH_OTHER, s, st);
        e = g_eval(h, s, Xw, ldxw, G, ldg, st);
    }
    if (owned) {
        hipError_t e2 = hipFreeAsync(work, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) rc = (e == hipErrorOutOfMemory) ? SHS_ERR_NOMEM : SHS_ERR_HIP;
    return rc;
}

int shs_solve_transposed_workspace(const shs_handle *h, int64_t s, int64_t r, size_t *bytes)
{
    if (!h) return -1;
    if (s < 0) return -2;
    if (r < 1) return -3;
    if (!bytes) return -4;
    TransLayout L;
    if (!trans_layout(h, s, r, &L)) return SHS_ERR_UNSUPPORTED;
    *bytes = L.total;
    return 0;
}

// The transposed solve after argument checks: right-hand sides D (r per
// shift), or, with chat set (r = 1), Ct^T c_j formed on the device.
static int transposed_impl(shs_handle *h, int64_t s, const double *shifts, int64_t r, const double *D, int64_t ldd,
                           const double *chat, int64_t ldc, int outputs, void *work, size_t work_bytes, double *X,
                           int64_t ldx, double *eta, int32_t *status, void *stream)
{
    const int64_t n = h->n, m = h->m;
    TransLayout L;
    if (!trans_layout(h, s, r, &L)) return SHS_ERR_UNSUPPORTED;
    if (L.nv > INT32_MAX / 64) return -2;
    hipStream_t st = (hipStream_t)stream;
    bool owned = false;
    if (work) {
        if (work_bytes < L.total) return -9;
    } else {
        RETURN_IF_HIP(hipMallocAsync(&work, L.total, st));
        owned = true;
    }
    hipError_t e = ensure_transposed(h, st);
    const int nv = (int)L.nv;
    double *shv = at<double>(work, L.shv), *E = at<double>(work, L.e), *Xv = at<double>(work, L.xv);
    int32_t *stv = at<int32_t>(work, L.stv);
    double *etav = at<double>(work, L.etav);
    const unsigned chunks = std::max<unsigned>(1, std::min<unsigned>(64, cdiv(n * m, 256 * 16)));
    if (e == hipSuccess) {
        if (chat) {   // r = 1: one item per shift, the shifts as given
            shv = const_cast<double *>(shifts);
            hipLaunchKernelGGL(tvec_pack_kernel, dim3((unsigned)nv, chunks), dim3(256), 0, st, (int)n, (int)m,
                               (int)h->p, (const double *)h->Ct, h->ldct, chat, ldc, E);
        } else {
            hipLaunchKernelGGL(transposed_pack_kernel, dim3((unsigned)nv, chunks), dim3(256), 0, st, (int)n,
                               (int)m, (int)r, (int)L.nch, shifts, D, ldd, shv, E);
        }
        e = hipGetLastError();
    }
    Geo g;
    geo(false, n, m, true, &g);
    if (e == hipSuccess) {
        SweepArgs<double> da{};
        da.n = (int)n;
        da.count = nv;
        da.H = h->Ht;
        da.ldh = h->ldh;
        da.shifts = shv;
        da.list = nullptr;
        da.Rtop = h->Rtop;
        da.E = E;
        da.e_stride = 2 * n * m;
        da.refl = at<double>(work, L.refl);
        da.refl_stride = L.refl_stride;
        da.Y = at<double>(work, L.yd);
        da.y_stride = 2 * n * m;
        da.status = stv;
        if (L.blocked) {
            const BlkBuf B{at<double>(work, L.zb), at<double>(work, L.bm), at<double>(work, L.m2),
                           at<double>(work, L.m2p), at<double>(work, L.m2q), L.blk_rows};
            e = sweep_blocked(h, nv, nullptr, nullptr, shv, B, da, st, E, h->Ht);
        } else {
            PhaseScope ps(h, PH_SWEEP, nv, st);
            if (!launch_sweep((int)m, true, da, st)) e = hipErrorInvalidValue;
        }
        QstarArgs<double> dq{};
        dq.n = (int)n;
        dq.count = nv;
        dq.list = nullptr;
        dq.refl = da.refl;
        dq.refl_stride = L.refl_stride;
        dq.tile_rows = g.g.tile_rows;
        dq.tile_stride = g.g.tile_stride;
        dq.slot = g.g.slot;
        dq.Y = da.Y;
        dq.y_stride = 2 * n * m;
        dq.X = Xv;
        dq.ldx = n;
        dq.accumulate = 0;
        if (e == hipSuccess) {
            PhaseScope ps(h, PH_QSTAR, nv, st);
            if (!launch_qstar((int)m, true, dq, st)) e = hipErrorInvalidValue;
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess && (outputs & SHS_OUT_ETA)) {
        // eta of the reversed system (Ht - sigma I) Z = J D, which is the
        // transposed system's: the residuals are J-permutations of each other
        // and ||Ht - sigma I||_inf = ||(H - sigma I)^T||_inf
        CertifyOpts co;
        co.H = h->Ht;
        co.offrow = h->ht_offrow;
        co.diag = h->ht_diag;
        co.nc = (int)m;
        co.E = E;
        co.lde = n;
        co.emax = at<unsigned long long>(work, L.emax);
        e = certify(h, nv, nullptr, nullptr, shv, Xv, n, nullptr, at<unsigned long long>(work, L.resmax),
                    at<unsigned long long>(work, L.xmax), etav, stv, nv, at<double>(work, L.xt), st, &co);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(transposed_unpack_kernel, dim3((unsigned)nv, chunks), dim3(256), 0, st, (int)n, (int)m,
                           (int)r, (int)L.nch, (const double *)Xv, (outputs & SHS_OUT_X) ? X : nullptr, ldx,
                           (outputs & SHS_OUT_ETA) ? (const double *)etav : nullptr, (const int32_t *)stv,
                           (outputs & SHS_OUT_ETA) ? eta : nullptr, status);
        e = hipGetLastError();
    }
    if (owned) {
        hipError_t e2 = hipFreeAsync(work, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return (e == hipErrorOutOfMemory) ? SHS_ERR_NOMEM : SHS_ERR_HIP;
    return 0;
}

int shs_solve_transposed(shs_handle *h, int64_t s, const double *shifts, int64_t r, const double *D, int64_t ldd,
                         int outputs, void *work, size_t work_bytes, double *X, int64_t ldx, double *eta,
                         int32_t *status, void *stream)
{
    if (!h) return -1;
    if (s < 0) return -2;
    if (s > 0 && !shifts) return -3;
    if (r < 1) return -4;
    if (s > 0 && !D) return -5;
    if (ldd < h->n) return -6;
    if (!(outputs & SHS_OUT_X) && !(outputs & SHS_OUT_ETA)) return -7;
    if (outputs & ~(SHS_OUT_X | SHS_OUT_ETA)) return -7;
    if (s == 0) return 0;
    if ((outputs & SHS_OUT_X) && (!X || ldx < h->n)) return -10;
    if ((outputs & SHS_OUT_ETA) && !eta) return -12;
    if (!status) return -13;
    return transposed_impl(h, s, shifts, r, D, ldd, nullptr, 0, outputs, work, work_bytes, X, ldx, eta, status,
                           stream);
}

int shs_solve_transposed_vec_workspace(const shs_handle *h, int64_t s, size_t *bytes)
{
    return shs_solve_transposed_workspace(h, s, 1, bytes);
}

int shs_solve_transposed_vec(shs_handle *h, int64_t s, const double *shifts, const double *chat, int64_t ldc,
                             int outputs, void *work, size_t work_bytes, double *X, int64_t ldx, double *eta,
                             int32_t *status, void *stream)
{
    if (!h) return -1;
    if (s < 0) return -2;
    if (s > 0 && !shifts) return -3;
    if (s > 0 && h->p > 0 && !chat) return -4;
    if (ldc < std::max<int64_t>(1, h->p)) return -5;
    if (!(outputs & SHS_OUT_X) && !(outputs & SHS_OUT_ETA)) return -6;
    if (outputs & ~(SHS_OUT_X | SHS_OUT_ETA)) return -6;
    if (s == 0) return 0;
    if ((outputs & SHS_OUT_X) && (!X || ldx < h->n)) return -9;
    if ((outputs & SHS_OUT_ETA) && !eta) return -11;
    if (!status) return -12;
    return transposed_impl(h, s, shifts, 1, nullptr, h->n, chat, ldc, outputs, work, work_bytes, X, ldx, eta,
                           status, stream);
}

int shs_solve_vec_workspace(const shs_handle *h, int64_t s, size_t *bytes)
{
    if (!h) return -1;
    if (s < 0) return -2;
    if (!bytes) return -3;
    VecLayout V;
    if (!vec_layout(h, s, &V)) return SHS_ERR_UNSUPPORTED;
    *bytes = V.total;
    return 0;
}

int shs_solve_vec(shs_handle *h, int64_t s, const double *shifts, const double *bhat, int64_t ldb, int outputs,
                  void *work, size_t work_bytes, double *X, int64_t ldx, double *eta, int32_t *status, void *stream)
{
    if (!h) return -1;
    if (s < 0 || s > INT32_MAX / 64) return -2;
    if (s > 0 && !shifts) return -3;
    if (s > 0 && !bhat) return -4;
    if (ldb < h->m) return -5;
    if (!(outputs & SHS_OUT_X) && !(outputs & SHS_OUT_ETA)) return -6;
    if (outputs & ~(SHS_OUT_X | SHS_OUT_ETA)) return -6;
    if (s == 0) return 0;
    if (!X || ldx < h->n) return -9;   // X is also the residual's input
    if ((outputs & SHS_OUT_ETA) && !eta) return -11;
    if (!status) return -12;
    const int64_t n = h->n, m = h->m;
    VecLayout V;
    if (!vec_layout(h, s, &V)) return SHS_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    if (h->timing) {
        h->marks.clear();
        h->last_mixed = false;
        h->tile_flops = h->update_flops = 0.0;
    }
    bool owned = false;
    if (work) {
        if (work_bytes < V.total) return -8;
    } else {
        RETURN_IF_HIP(hipMallocAsync(&work, V.total, st));
        owned = true;
    }
    const Layout &L = V.base;
    double *Xm = at<double>(work, L.x);   // Q* output, m columns per shift (the first one nonzero)
    hipError_t e = solve_fp64(h, s, nullptr, nullptr, shifts, work, L, Xm, n, status, st, bhat, ldb);
    const bool want_eta = outputs & SHS_OUT_ETA;
    double *E = want_eta ? at<double>(work, V.e) : nullptr;
    if (e == hipSuccess) {
        PhaseScope ps(h, PH_OTHER, s, st);
        hipLaunchKernelGGL(vec_out_kernel, dim3((unsigned)s, std::max<unsigned>(1, std::min<unsigned>(16, cdiv(n, 256)))),
                           dim3(256), 0, st, (int)n, (int)m, (const double *)Xm, X, ldx, (const double *)h->Rtop,
                           bhat, ldb, E);
        e = hipGetLastError();
    }
    if (e == hipSuccess && want_eta) {
        CertifyOpts co;
        co.nc = 1;
        co.E = E;
        co.lde = n;
        co.emax = at<unsigned long long>(work, V.emax);
        e = certify(h, s, nullptr, nullptr, shifts, X, ldx, nullptr, at<unsigned long long>(work, L.resmax),
                    at<unsigned long long>(work, L.xmax), eta, status, s, at<double>(work, L.xt), st, &co);
    }
    if (owned) {
        hipError_t e2 = hipFreeAsync(work, st);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return (e == hipErrorOutOfMemory) ? SHS_ERR_NOMEM : SHS_ERR_HIP;
    return 0;
}

int shs_apply_q(const shs_handle *h, int64_t ncols, const double *Xred, int64_t ld, double *Xorig, int64_t ldo,
                void *stream)
{
    if (!h) return -1;
    if (ncols < 0) return -2;
    if (ncols > 0 && !Xred) return -3;
    if (ld < h->n) return -4;
    if (ncols > 0 && !Xorig) return -5;
    if (ldo < h->n) return -6;
    if (ncols == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n, m = h->m;
    if (Xorig != Xred || ld != ldo)
        hipLaunchKernelGGL(copy_complex_kernel, dim3(cdiv(n * ncols, 256)), dim3(256), 0, st, (int)n, (int)ncols,
                           Xred, ld, Xorig, ldo);
    // Q = Q_B Q_A S: X <- S X, then the Q_A reflectors last to first, then Q_B's
    hipLaunchKernelGGL(scale_rows_complex_kernel, dim3(cdiv(n * ncols, 256)), dim3(256), 0, st, (int)n,
                       (int)ncols, Xorig, ldo, (const double *)h->sgn);
    if (h->nrefl < kApplyQBlock || ncols > INT32_MAX / 2) {
        // a few reflectors: one launch each
        for (int64_t idx = h->nrefl - 1; idx >= 0; --idx) {
            const int64_t r0 = refl_start(m, idx);
            const int64_t L = n - r0;
            hipLaunchKernelGGL(reflect_complex_kernel, dim3((unsigned)ncols), dim3(256), 0, st, (int)L, (int)r0,
                               Xorig, ldo, (const double *)(h->V + idx * n + r0), (const double *)(h->tauv + idx));
        }
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? 0 : SHS_ERR_HIP;
    }
    // blocks of kApplyQBlock reflectors as I - V T V^T (compact WY), applied
    // last block first with FP64 matrix-core GEMMs on the real and imaginary
    // parts of X side by side
    const int64_t nb = kApplyQBlock, nc2 = 2 * ncols;
    const size_t part_elems = (size_t)1 << 22;
    const size_t bytes = sizeof(double) * ((size_t)n * nc2 + 3 * nb * nb + 2 * nb * nc2 + part_elems);
    void *work = nullptr;
    RETURN_IF_HIP(hipMallocAsync(&work, bytes, st));
    double *Xr = static_cast<double *>(work);
    double *G = Xr + (size_t)n * nc2, *T = G + nb * nb, *W = T + nb * nb, *W2 = W + nb * nc2, *part = W2 + nb * nc2;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(split_complex_kernel, dim3(cdiv(n, 256), (unsigned)ncols), dim3(256), 0, st, (int)n,
                       (const double *)Xorig, ldo, Xr, (int)ncols);
    for (int64_t j0 = (h->nrefl - 1) / nb * nb; j0 >= 0 && e == hipSuccess; j0 -= nb) {
        // reflector idx starts at row refl_start(m, idx) = idx, so columns
        // j0 .. j0+bb-1 of V are zero above row j0 + (column - j0)
        const int bb = (int)std::min<int64_t>(nb, h->nrefl - j0);
        const int L = (int)(n - j0);
        const double *Vb = h->V + j0 * n + j0;
        e = gemm_f64(true, false, bb, bb, L, 1.0, Vb, n, Vb, n, G, nb, false, part, part_elems, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(wy_t_kernel, dim3(1), dim3(nb), 0, st, bb, (const double *)G, (int)nb,
                               (const double *)(h->tauv + j0), T);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = gemm_f64(true, false, bb, (int)nc2, L, 1.0, Vb, n, Xr + j0, n, W, nb, false, part, part_elems, st);
        if (e == hipSuccess)
            e = gemm_f64(false, false, bb, (int)nc2, bb, 1.0, T, nb, W, nb, W2, nb, false, nullptr, 0, st);
        if (e == hipSuccess)
            e = gemm_f64(false, false, L, (int)nc2, bb, -1.0, Vb, n, W2, nb, Xr + j0, n, true, nullptr, 0, st);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(join_complex_kernel, dim3(cdiv(n, 256), (unsigned)ncols), dim3(256), 0, st, (int)n,
                           (const double *)Xr, (int)ncols, Xorig, ldo);
        e = hipGetLastError();
    }
    const hipError_t e2 = hipFreeAsync(work, st);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return (e == hipErrorOutOfMemory) ? SHS_ERR_NOMEM : SHS_ERR_HIP;
    return 0;
}

int shs_get_reduced(const shs_handle *h, double *H, int64_t ldh, double *R, int64_t ldr, double *Ct,
                    int64_t ldct, void *stream)
{
    if (!h) return -1;
    if (H && ldh < h->n) return -3;
    if (R && ldr < h->n) return -5;
    if (Ct && ldct < std::max<int64_t>(1, h->p)) return -7;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n, m = h->m, p = h->p;
    if (H) RETURN_IF_HIP(hipMemcpy2DAsync(H, sizeof(double) * ldh, h->H, sizeof(double) * h->ldh,
                                          sizeof(double) * n, n, hipMemcpyDeviceToDevice, st));
    if (R) RETURN_IF_HIP(hipMemcpy2DAsync(R, sizeof(double) * ldr, h->Bw, sizeof(double) * n, sizeof(double) * n, m,
                                          hipMemcpyDeviceToDevice, st));
    if (Ct && p > 0)
        RETURN_IF_HIP(hipMemcpy2DAsync(Ct, sizeof(double) * ldct, h->Ct, sizeof(double) * h->ldct,
                                       sizeof(double) * p, n, hipMemcpyDeviceToDevice, st));
    return 0;
}

int shs_info(const shs_handle *h, shs_info_t *info)
{
    if (!h) return -1;
    if (!info) return -2;
    info->n = h->n;
    info->m = h->m;
    info->p = h->p;
    info->reduce_ms = h->reduce_ms;
    info->resident_bytes = h->resident;
    return 0;
}

int shs_set_timing(shs_handle *h, int enable)
{
    if (!h) return -1;
    h->timing = enable != 0;
    h->marks.clear();
    return 0;
}

int shs_last_timings(const shs_handle *h, shs_timings_t *out)
{
    if (!h) return -1;
    if (!out) return -2;
    std::memset(out, 0, sizeof(*out));
    if (!h->marks.empty()) RETURN_IF_HIP(hipEventSynchronize(h->marks.back().b));
    double *ms[PH_COUNT] = {&out->sweep_ms,       &out->qstar_ms,        &out->residual_ms,
                            &out->sweep32_ms,     &out->sweep32_dense_ms, &out->other_ms,
                            &out->sweep_tile_ms,  &out->sweep_update_ms};
    int64_t *calls[PH_COUNT] = {&out->sweep_calls,      &out->qstar_calls,         &out->residual_calls,
                                &out->sweep32_calls,    &out->sweep32_dense_calls, &out->other_calls,
                                &out->sweep_tile_calls, &out->sweep_update_calls};
    for (const auto &mk : h->marks) {
        float t = 0.f;
        RETURN_IF_HIP(hipEventElapsedTime(&t, mk.a, mk.b));
        *ms[mk.phase] += t;
        *calls[mk.phase] += 1;
        if (mk.phase == PH_SWEEP) out->sweep_shifts += mk.shifts;
        if (mk.phase == PH_SWEEP32) out->sweep32_shifts += mk.shifts;
    }
    if (h->last_mixed) {
        // the mixed mode counts its rounds and shifts on the device
        long long st[3] = {0, 0, 0};
        RETURN_IF_HIP(hipMemcpy(st, h->dstats, sizeof(st), hipMemcpyDeviceToHost));
        out->refine_iterations = st[0];
        out->fallback_shifts = st[1];
        out->sweep32_dense_shifts = st[2];
    }
    out->sweep_tile_flops = h->tile_flops;
    out->sweep_update_flops = h->update_flops;
    return 0;
}

void shs_destroy(shs_handle *h)
{
    if (!h) return;
    int dev = 0;
    hipGetDevice(&dev);
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    free_handle(h);
    hipSetDevice(dev);
}

}  // extern "C"
