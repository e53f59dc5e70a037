// Shared device/host helpers of the shiftsolve library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace shs {

constexpr int kWave = 64;

// Per-shift reflector-store slot, in elements of the sweep precision:
//   [tau, pad, v_0.re, v_0.im, ..., v_{m-1}.re, v_{m-1}.im]            structured
//   [..., y_0.re, y_0.im, ..., y_{m-1}.re, y_{m-1}.im]                  + dense RHS
// The implicit last entry v_m of every reflector is 1.
__host__ __device__ constexpr int slot_elems(int m, bool dense) { return 2 + 2 * m + (dense ? 2 * m : 0); }

// Packed solutions of the residual GEMM: rows up to a whole chunk of 16,
// row stride (in doubles) for `cols` complex columns up to a whole tile of 64.
__host__ __device__ inline int64_t residual_pack_rows(int64_t n) { return (n + 15) / 16 * 16; }
__host__ __device__ inline int64_t residual_pack_ld(int64_t cols) { return (cols + 63) / 64 * 128; }

// Rows of the window a lane keeps in registers: the state of one row is
// 2(m+1) values (+2m for a dense right-hand side); the budget keeps the
// kernel near 200 VGPRs so that two waves fit on each SIMD.
template <typename T, int M, bool DENSE>
__host__ __device__ constexpr int rows_per_lane()
{
    constexpr int vals = 2 * (M + 1) + (DENSE ? 2 * M : 0);
    constexpr int vgprs = vals * (int)(sizeof(T) / 4);
    constexpr int r = 144 / vgprs;
    // FP32 windows of m >= 13: the step's temporaries (pivot row, reflector,
    // dense right-hand side) grow with m as well, and with the budget above
    // the kernels spill hundreds of bytes per lane; fewer row slots remove
    // most of it (the m = 16 mixed solve at n = 8192 runs 25% faster)
    if (sizeof(T) == 4 && M >= 13) return DENSE ? 1 : 2;
    return r < 1 ? 1 : (r > 8 ? 8 : r);
}

__device__ inline double readlane(double x, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

__device__ inline float readlane(float x, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

template <typename T> __device__ inline T dsqrt(T x);
template <> __device__ inline double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ inline float dsqrt<float>(float x) { return sqrtf(x); }

// 1/x and 1/sqrt(x) from the hardware estimates refined by Newton steps
// (two in FP64, one in FP32): within an ulp or two, not correctly rounded,
// and cheaper than the division and square root sequences.  For normal
// positive x (the callers guard zero).
template <typename T> __device__ inline T rcp_nr(T x);
template <> __device__ inline double rcp_nr<double>(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
template <> __device__ inline float rcp_nr<float>(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
template <typename T> __device__ inline T rsq_nr(T x);
template <> __device__ inline double rsq_nr<double>(double x)
{
    // y <- y + y (1 - x y^2) / 2
    const double h = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return fma(y, fma(-h * y, y, 0.5), y);
}
template <> __device__ inline float rsq_nr<float>(float x)
{
    const float h = 0.5f * x;
    const float y = __builtin_amdgcn_rsqf(x);
    return fmaf(y, fmaf(-h * y, y, 0.5f), y);
}

// Non-negative doubles order like their bit patterns, which lets an
// unsigned 64-bit atomic max act as a floating-point max.
__device__ inline void atomic_max_nonneg(unsigned long long *addr, double v)
{
    atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

}  // namespace shs

#define SHS_HIP_CHECK(expr)                                                      \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            fprintf(stderr, "shiftsolve: %s failed: %s (%s:%d)\n", #expr,        \
                    hipGetErrorString(e_), __FILE__, __LINE__);                  \
            return SHS_ERR_HIP;                                                  \
        }                                                                        \
    } while (0)
