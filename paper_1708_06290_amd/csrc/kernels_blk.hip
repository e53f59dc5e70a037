// Instances of the blocked FP64 sweep kernels (row-tile reflectors + block
// transform, and the all-shift update GEMM) for m = 1 .. 16 with the
// structured right-hand side (the dense one: kernels_blk_dense.hip).
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
    if (dense) return launch_blk_tri_dense(m, a, st);
    bool ok = false;
    SHS_DISPATCH_M(m, {
        hipLaunchKernelGGL((blk_tri_kernel<double, MM, false>), dim3(a.count), dim3(kWave), 0, st, a);
        ok = true;
    });
    return ok;
}

bool launch_zupd(int m, const ZupdArgsT<double> &a, hipStream_t st)
{
    if (a.lo <= a.r0) return true;
    if (!zupd_args_ok(m, a)) return false;
    const int w = blk_cols(m, a.nr != 0);
    const dim3 grid((unsigned)((a.ncols / zupd_bn(w)) * ((a.lo - a.r0 + 127) / 128)));
    switch (w) {
    case 2: hipLaunchKernelGGL((zupd_kernel<2>), grid, dim3(256), kZupdLds, st, a); return true;
    case 4: hipLaunchKernelGGL((zupd_kernel<4>), grid, dim3(256), kZupdLds, st, a); return true;
    case 8: hipLaunchKernelGGL((zupd_kernel<8>), grid, dim3(256), kZupdLds, st, a); return true;
    case 16: hipLaunchKernelGGL((zupd_kernel<16>), grid, dim3(256), kZupdLds, st, a); return true;
    case 24: hipLaunchKernelGGL((zupd_kernel<24>), grid, dim3(256), kZupdLds, st, a); return true;
    case 32: hipLaunchKernelGGL((zupd_kernel<32>), grid, dim3(256), kZupdLds, st, a); return true;
    case 48: hipLaunchKernelGGL((zupd_kernel<48>), grid, dim3(256), kZupdLds, st, a); return true;
    case 64: hipLaunchKernelGGL((zupd_kernel<64>), grid, dim3(256), kZupdLds, st, a); return true;
    default: return false;
    }
}

}  // namespace shs
