// Instances of the blocked FP64 sweep kernels (row-tile reflectors + block
// transform, and the all-shift update GEMM) for m = 1 .. 16, with the
// structured right-hand side, and with a dense one for m = 1 .. 8.
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool blk_geometry(bool fp32, int m, bool dense, int *tile_rows, int *width)
{
    if (dense && m > kBlkDenseMaxM) return false;
    bool ok = false;
    SHS_DISPATCH_M(m, {
        if (fp32)
            *tile_rows = dense ? kWave * blk_rb<float, MM, true>() : kWave * blk_rb<float, MM, false>();
        else
            *tile_rows = dense ? kWave * blk_rb<double, MM, true>() : kWave * blk_rb<double, MM, false>();
        *width = blk_cols(MM, dense);
        ok = true;
    });
    return ok;
}

bool launch_blk_tri(int m, bool dense, const BlkTriArgsT<double> &a, hipStream_t st)
{
    bool ok = false;
    if (!dense) {
        SHS_DISPATCH_M(m, {
            hipLaunchKernelGGL((blk_tri_kernel<double, MM, false>), dim3(a.count), dim3(kWave), 0, st, a);
            ok = true;
        });
    } else {
        switch (m) {
        case 1: hipLaunchKernelGGL((blk_tri_kernel<double, 1, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 2: hipLaunchKernelGGL((blk_tri_kernel<double, 2, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 3: hipLaunchKernelGGL((blk_tri_kernel<double, 3, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 4: hipLaunchKernelGGL((blk_tri_kernel<double, 4, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 5: hipLaunchKernelGGL((blk_tri_kernel<double, 5, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 6: hipLaunchKernelGGL((blk_tri_kernel<double, 6, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 7: hipLaunchKernelGGL((blk_tri_kernel<double, 7, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 8: hipLaunchKernelGGL((blk_tri_kernel<double, 8, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        default: return false;
        }
    }
    return ok;
}

// What the direct-to-LDS loads assume: 16-byte aligned groups of rows of H
// and of columns of Bm (two doubles or four floats), at least one group of
// rows, K a whole number of chunks unless the padding rows of Bm are zero
// (the bottom tile).
template <typename T>
static bool zupd_args_ok(int m, const ZupdArgsT<T> &a)
{
    constexpr int G = 16 / (int)sizeof(T);
    return !((a.r0 | a.lo) % G || a.lo - a.r0 < G || a.ldh % G || a.ldb % G || a.ncols % 128 != 0 || a.c0 < 0 ||
             (a.has_zin && a.K % 16 != 0 && a.nr == 0) || a.K <= 0 || a.n < a.lo ||
             ((uintptr_t)a.H | (uintptr_t)a.Bm) & 15 || (a.nr != 0 && a.nr != m));
}

bool launch_zupd(int m, const ZupdArgsT<double> &a, hipStream_t st)
{
    if (a.lo <= a.r0) return true;
    if (!zupd_args_ok(m, a)) return false;
    const dim3 grid((unsigned)((a.ncols / 128) * ((a.lo - a.r0 + 127) / 128)));
    switch (blk_cols(m, a.nr != 0)) {
    case 2: hipLaunchKernelGGL((zupd_kernel<2>), grid, dim3(256), kZupdLds, st, a); return true;
    case 4: hipLaunchKernelGGL((zupd_kernel<4>), grid, dim3(256), kZupdLds, st, a); return true;
    case 8: hipLaunchKernelGGL((zupd_kernel<8>), grid, dim3(256), kZupdLds, st, a); return true;
    case 16: hipLaunchKernelGGL((zupd_kernel<16>), grid, dim3(256), kZupdLds, st, a); return true;
    case 32: hipLaunchKernelGGL((zupd_kernel<32>), grid, dim3(256), kZupdLds, st, a); return true;
    default: return false;
    }
}

bool launch_zupd(int m, const ZupdArgsT<float> &a, hipStream_t st)
{
    if (a.lo <= a.r0) return true;
    if (!zupd_args_ok(m, a)) return false;
    const dim3 grid((unsigned)((a.ncols / 128) * ((a.lo - a.r0 + 127) / 128)));
    switch (blk_cols(m, a.nr != 0)) {
    case 2: hipLaunchKernelGGL((zupd32_kernel<2>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 4: hipLaunchKernelGGL((zupd32_kernel<4>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 8: hipLaunchKernelGGL((zupd32_kernel<8>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 16: hipLaunchKernelGGL((zupd32_kernel<16>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 32: hipLaunchKernelGGL((zupd32_kernel<32>), grid, dim3(256), kZupd32Lds, st, a); return true;
    default: return false;
    }
}

}  // namespace shs
