// Instances of the blocked FP64 sweep kernels (row-tile reflectors + block
// transform, and the all-shift update GEMM) for m = 1 .. 16.
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool blk_geometry(int m, int *tile_rows, int *width)
{
    bool ok = false;
    SHS_DISPATCH_M(m, {
        *tile_rows = SweepShape<double, MM, false>::TT;
        *width = blk_width(MM);
        ok = true;
    });
    return ok;
}

bool launch_blk_tri(int m, const BlkTriArgs &a, hipStream_t st)
{
    bool ok = false;
    SHS_DISPATCH_M(m, {
        hipLaunchKernelGGL((blk_tri_kernel<MM>), dim3(a.count), dim3(kWave), 0, st, a);
        ok = true;
    });
    return ok;
}

bool launch_zupd(int m, const ZupdArgs &a, hipStream_t st)
{
    if (a.lo <= a.r0) return true;
    // what the direct-to-LDS loads assume: 16-byte aligned pairs of rows of
    // H and of columns of Bm, at least two rows, K a whole number of chunks
    // unless the padding rows of Bm are zero (the bottom tile)
    if ((a.r0 | a.lo) & 1 || a.lo - a.r0 < 2 || a.ldh & 1 || a.ldb & 1 || a.ncols % 128 != 0 || a.c0 < 0 ||
        (a.has_zin && a.K % 16 != 0) || a.K <= 0 || a.n < a.lo || ((uintptr_t)a.H | (uintptr_t)a.Bm) & 15)
        return false;
    const dim3 grid((unsigned)((a.ncols / 128) * ((a.lo - a.r0 + 127) / 128)));
    switch (blk_width(m)) {
    case 2: hipLaunchKernelGGL((zupd_kernel<2>), grid, dim3(256), kZupdLds, st, a); return true;
    case 4: hipLaunchKernelGGL((zupd_kernel<4>), grid, dim3(256), kZupdLds, st, a); return true;
    case 8: hipLaunchKernelGGL((zupd_kernel<8>), grid, dim3(256), kZupdLds, st, a); return true;
    case 16: hipLaunchKernelGGL((zupd_kernel<16>), grid, dim3(256), kZupdLds, st, a); return true;
    case 32: hipLaunchKernelGGL((zupd_kernel<32>), grid, dim3(256), kZupdLds, st, a); return true;
    default: return false;
    }
}

}  // namespace shs
