// General FP64 GEMM on the matrix cores: C = alpha * op(A) * op(B) (+ C).
//
// Column-major operands; op(A) is M x K, op(B) is K x N.  Used by the
// blocked controller-Hessenberg reduction for its trailing updates and
// block-reflector products, whose shapes range from square to tall-skinny
// (N = m columns, K = n) and short-wide (M = p rows).  A workgroup of 4 waves
// computes a BM x BN tile of C from K-chunks of 16 staged in LDS, as
// 16 x 16 tiles of v_mfma_f64_16x16x4f64 (lane l holds A(l%16, l/16) and
// B(l/16, l%16); result register r of lane l is D(4 r + l/16, l%16)).
// Out-of-range rows, columns and k are zero-filled, so any shape is
// accepted.  A long K is split over gridDim.z workgroups whose partial tiles
// go to a workspace and are summed in a fixed order by a second kernel, so
// the result does not depend on scheduling.
#pragma once

#include <algorithm>
#include <cstdio>
#include <vector>

#include "common.hpp"

namespace shs {

// Grid of one GEMM launch: gx x gy tiles of BM x BN, K split into nsplit
// chunks of kchunk (a multiple of 16).  K is split when the tile grid alone
// cannot fill the chip: aim at ~1024 workgroups, chunks of at least 128,
// partials within the workspace (part_elems doubles).
struct GemmPlan {
    int gx, gy, nsplit, kchunk;
};

inline GemmPlan gemm_plan(int M, int N, int K, int BM, int BN, bool has_part, size_t part_elems)
{
    GemmPlan g;
    g.gx = (M + BM - 1) / BM;
    g.gy = (N + BN - 1) / BN;
    g.nsplit = 1;
    const int64_t tiles = (int64_t)g.gx * g.gy;
    if (tiles < 512 && K >= 256 && has_part) {
        int64_t want = std::min<int64_t>(1024 / tiles, K / 128);
        const int64_t room = (int64_t)(part_elems / ((size_t)M * N));
        g.nsplit = (int)std::max<int64_t>(1, std::min(want, room));
    }
    g.kchunk = 16;
    if (K > 0) {
        g.kchunk = ((K + g.nsplit - 1) / g.nsplit + 15) / 16 * 16;
        g.nsplit = (K + g.kchunk - 1) / g.kchunk;
    }
    return g;
}

// Tile shape gemm_shape picks for an M x N result.
inline void gemm_tile(int M, int N, int *BM, int *BN)
{
    if (N <= 16 && M <= 64) { *BM = 64; *BN = 16; }
    else if (N <= 16) { *BM = 256; *BN = 16; }
    else if (M <= 16) { *BM = 16; *BN = 256; }
    else if (M <= 64) { *BM = 64; *BN = 128; }
    else { *BM = 128; *BN = 128; }
}

// Dry run of a sequence of launches: instead of launching, every GEMM is
// checked against the device regions registered here (base address and
// size in doubles): the extent each operand is read or written over, the
// split-K partials against the workspace, the grid against the launch
// limits, and that the result does not overlap an operand.  Used on the
// host to validate a whole launch plan without a GPU.
struct LaunchCheck {
    struct Region { uintptr_t lo, hi; const char *name; };
    std::vector<Region> regions;
    int64_t launches = 0, violations = 0;
    char first[256] = {0};

    void add(const void *p, size_t elems, const char *name)
    {
        const uintptr_t lo = (uintptr_t)p;
        regions.push_back({lo, lo + elems * sizeof(double), name});
    }
    void fail(const char *what, int M, int N, int K)
    {
        if (violations++ == 0) snprintf(first, sizeof(first), "%s (M=%d N=%d K=%d)", what, M, N, K);
    }
    // [p, p + last] (last in doubles, inclusive) inside one region
    const Region *inside(const double *p, int64_t last) const
    {
        const uintptr_t lo = (uintptr_t)p, hi = lo + (uintptr_t)(last + 1) * sizeof(double);
        for (const auto &r : regions)
            if (lo >= r.lo && hi <= r.hi) return &r;
        return nullptr;
    }
    void gemm(bool ta, bool tb, int M, int N, int K, const double *A, int64_t lda, const double *B, int64_t ldb,
              const double *C, int64_t ldc, const double *part, size_t part_elems)
    {
        ++launches;
        int BM = 0, BN = 0;
        gemm_tile(M, N, &BM, &BN);
        const GemmPlan g = gemm_plan(M, N, K, BM, BN, part != nullptr, part_elems);
        if (g.gx < 1 || g.gy < 1 || g.gy > 65535 || g.nsplit < 1 || g.nsplit > 65535) fail("grid", M, N, K);
        if ((int64_t)g.nsplit * g.kchunk < K || (int64_t)(g.nsplit - 1) * g.kchunk >= std::max(K, 1))
            fail("k split", M, N, K);
        if (g.nsplit > 1 && (!part || (size_t)g.nsplit * M * N > part_elems)) fail("split-K partials", M, N, K);
        // extents: op(A) is M x K, op(B) is K x N, C is M x N (column-major)
        if (K > 0) {
            if ((ta ? lda < K : lda < M) || !inside(A, ta ? (int64_t)(M - 1) * lda + K - 1
                                                           : (int64_t)(K - 1) * lda + M - 1))
                fail("A extent", M, N, K);
            if ((tb ? ldb < N : ldb < K) || !inside(B, tb ? (int64_t)(K - 1) * ldb + N - 1
                                                           : (int64_t)(N - 1) * ldb + K - 1))
                fail("B extent", M, N, K);
        }
        const int64_t clast = (int64_t)(N - 1) * ldc + M - 1;
        if (ldc < M || !inside(C, clast)) fail("C extent", M, N, K);
        auto overlap = [&](const double *X, int64_t xlast) {
            const uintptr_t a0 = (uintptr_t)C, a1 = a0 + (uintptr_t)(clast + 1) * 8;
            const uintptr_t b0 = (uintptr_t)X, b1 = b0 + (uintptr_t)(xlast + 1) * 8;
            return a0 < b1 && b0 < a1;
        };
        if (K > 0 && (overlap(A, ta ? (int64_t)(M - 1) * lda + K - 1 : (int64_t)(K - 1) * lda + M - 1) ||
                      overlap(B, tb ? (int64_t)(K - 1) * ldb + N - 1 : (int64_t)(N - 1) * ldb + K - 1)))
            fail("result overlaps an operand", M, N, K);
        if (g.nsplit > 1 && part && overlap(part, (int64_t)g.nsplit * M * N - 1)) fail("partials overlap C", M, N, K);
    }
};

typedef double gemm_dbl4 __attribute__((ext_vector_type(4)));

// WM waves along M, 4 / WM along N; each wave owns (BM / WM) x (BN / (4 / WM)).
template <bool TA, bool TB, int BM, int BN, int WM>
__global__ __launch_bounds__(256) void gemm_f64_kernel(int M, int N, int K, int kchunk, double alpha,
                                                       const double *A, int64_t lda, const double *B, int64_t ldb,
                                                       double *C, int64_t ldc, int accumulate, double *part)
{
    constexpr int BK = 16, WN = 4 / WM;
    constexpr int TM = BM / (WM * 16), TN = BN / (WN * 16);
    constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
    static_assert(TM >= 1 && TN >= 1 && EA >= 1 && EB >= 1, "tile shape");
    __shared__ double As[BK][BM];
    __shared__ double Bs[BK][BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);

    gemm_dbl4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = gemm_dbl4{0.0, 0.0, 0.0, 0.0};

    double ra[EA], rb[EB];
    // op(A)(i, k) = TA ? A[k + i lda] : A[i + k lda]; the contiguous index
    // runs fastest over the threads.
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            int i, k;
            if (TA) { k = k0 + (tid % BK); i = i0 + tid / BK + (256 / BK) * e; }
            else    { i = i0 + (tid % BM); k = k0 + tid / BM + (256 / BM) * e; }
            const bool ok = i < M && k < ke;
            ra[e] = ok ? (TA ? A[(int64_t)i * lda + k] : A[(int64_t)k * lda + i]) : 0.0;
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            int j, k;
            if (TB) { j = j0 + (tid % BN); k = k0 + tid / BN + (256 / BN) * e; }
            else    { k = k0 + (tid % BK); j = j0 + tid / BK + (256 / BK) * e; }
            const bool ok = j < N && k < ke;
            rb[e] = ok ? (TB ? B[(int64_t)k * ldb + j] : B[(int64_t)j * ldb + k]) : 0.0;
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            if (TA) As[tid % BK][tid / BK + (256 / BK) * e] = ra[e];
            else    As[tid / BM + (256 / BM) * e][tid % BM] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            if (TB) Bs[tid / BN + (256 / BN) * e][tid % BN] = rb[e];
            else    Bs[tid % BK][tid / BK + (256 / BK) * e] = rb[e];
        }
    };

    if (kb < ke) gload(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (k0 + BK < ke) gload(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[TM], bf[TN];
#pragma unroll
            for (int mt = 0; mt < TM; ++mt) af[mt] = As[kk + lane / 16][(wm * TM + mt) * 16 + lane % 16];
#pragma unroll
            for (int nt = 0; nt < TN; ++nt) bf[nt] = Bs[kk + lane / 16][(wn * TN + nt) * 16 + lane % 16];
#pragma unroll
            for (int mt = 0; mt < TM; ++mt)
#pragma unroll
                for (int nt = 0; nt < TN; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mt], bf[nt], acc[mt][nt], 0, 0, 0);
        }
    }
    const bool split = gridDim.z > 1;
#pragma unroll
    for (int mt = 0; mt < TM; ++mt)
#pragma unroll
        for (int nt = 0; nt < TN; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + (wm * TM + mt) * 16 + 4 * r + lane / 16;
                const int j = j0 + (wn * TN + nt) * 16 + lane % 16;
                if (i < M && j < N) {
                    if (split) {
                        part[((int64_t)blockIdx.z * N + j) * M + i] = acc[mt][nt][r];
                    } else {
                        double *pc = C + (int64_t)j * ldc + i;
                        *pc = accumulate ? fma(alpha, acc[mt][nt][r], *pc) : alpha * acc[mt][nt][r];
                    }
                }
            }
}

// C(i, j) = alpha * sum_z part[z][j][i] (+ C(i, j)), z in increasing order.
__global__ __launch_bounds__(256) void gemm_splitk_sum_kernel(int M, int N, int nsplit, double alpha,
                                                              const double *part, double *C, int64_t ldc,
                                                              int accumulate)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t MN = (int64_t)M * N;
    if (idx >= MN) return;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[z * MN + idx];
    const int64_t j = idx / M, i = idx % M;
    double *pc = C + j * ldc + i;
    *pc = accumulate ? fma(alpha, s, *pc) : alpha * s;
}

template <bool TA, bool TB, int BM, int BN, int WM>
inline void gemm_launch(int M, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                        int64_t ldb, double *C, int64_t ldc, int acc, double *part, size_t part_elems,
                        hipStream_t st)
{
    const GemmPlan g = gemm_plan(M, N, K, BM, BN, part != nullptr, part_elems);
    const int gx = g.gx, gy = g.gy, nsplit = g.nsplit, kchunk = g.kchunk;
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, BM, BN, WM>), dim3(gx, gy, nsplit), dim3(256), 0, st, M, N, K,
                       kchunk, alpha, A, lda, B, ldb, C, ldc, acc, part);
    if (nsplit > 1) {
        const int64_t MN = (int64_t)M * N;
        hipLaunchKernelGGL(gemm_splitk_sum_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, M, N,
                           nsplit, alpha, (const double *)part, C, ldc, acc);
    }
}

template <bool TA, bool TB>
inline void gemm_shape(int M, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *C, int64_t ldc, int acc, double *part, size_t part_elems,
                       hipStream_t st)
{
    int BM = 0, BN = 0;
    gemm_tile(M, N, &BM, &BN);
    if (BM == 64 && BN == 16)
        gemm_launch<TA, TB, 64, 16, 4>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else if (BM == 256)
        gemm_launch<TA, TB, 256, 16, 4>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else if (BM == 16)
        gemm_launch<TA, TB, 16, 256, 1>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else if (BM == 64)
        gemm_launch<TA, TB, 64, 128, 4>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else
        gemm_launch<TA, TB, 128, 128, 2>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
}

// C = alpha op(A) op(B) (+ C when accumulate).  With K = 0 an overwrite
// still zeroes C; an empty C is a no-op.  part (part_elems doubles, may be
// null) is the split-K workspace; it must not overlap the operands.
inline hipError_t gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int64_t lda,
                           const double *B, int64_t ldb, double *C, int64_t ldc, bool accumulate, double *part,
                           size_t part_elems, hipStream_t st, LaunchCheck *chk = nullptr)
{
    if (M <= 0 || N <= 0 || (K <= 0 && accumulate)) return hipSuccess;
    if (chk) {   // dry run: validate, launch nothing
        chk->gemm(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, part, part_elems);
        return hipSuccess;
    }
    const int acc = accumulate ? 1 : 0;
    if (!ta && !tb) gemm_shape<false, false>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else if (!ta && tb) gemm_shape<false, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else if (ta && !tb) gemm_shape<true, false>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    else gemm_shape<true, true>(M, N, K, alpha, A, lda, B, ldb, C, ldc, acc, part, part_elems, st);
    return hipGetLastError();
}

}  // namespace shs
