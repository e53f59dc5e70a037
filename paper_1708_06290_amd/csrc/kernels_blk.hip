// Instances of the blocked FP64 sweep kernels (row-tile reflectors + block
// transform, and the all-shift update GEMM) for m = 1 .. 16, with the
// structured right-hand side, and with a dense one for m = 1 .. 8.
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool blk_geometry(int m, bool dense, int *tile_rows, int *width)
{
    if (dense && m > kBlkDenseMaxM) return false;
    bool ok = false;
    SHS_DISPATCH_M(m, {
        *tile_rows = dense ? SweepShape<double, MM, true>::TT : SweepShape<double, MM, false>::TT;
        *width = blk_cols(MM, dense);
        ok = true;
    });
    return ok;
}

bool launch_blk_tri(int m, bool dense, const BlkTriArgs &a, hipStream_t st)
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

bool launch_zupd(int m, const ZupdArgs &a, hipStream_t st)
{
    if (a.lo <= a.r0) return true;
    // what the direct-to-LDS loads assume: 16-byte aligned pairs of rows of
    // H and of columns of Bm, at least two rows, K a whole number of chunks
    // unless the padding rows of Bm are zero (the bottom tile)
    if ((a.r0 | a.lo) & 1 || a.lo - a.r0 < 2 || a.ldh & 1 || a.ldb & 1 || a.ncols % 128 != 0 || a.c0 < 0 ||
        (a.has_zin && a.K % 16 != 0 && a.nr == 0) || a.K <= 0 || a.n < a.lo ||
        ((uintptr_t)a.H | (uintptr_t)a.Bm) & 15 || (a.nr != 0 && a.nr != m))
        return false;
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

}  // namespace shs
