// Instances of the blocked FP32 tile kernel with a dense right-hand side (the
// mixed form's corrections), m = 1 .. 16, and of the FP32 update GEMM.
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool launch_blk_tri_dense(int m, const BlkTriArgsT<float> &a, hipStream_t st)
{
    switch (m) {
    case 1: hipLaunchKernelGGL((blk_tri_kernel<float, 1, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 2: hipLaunchKernelGGL((blk_tri_kernel<float, 2, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 3: hipLaunchKernelGGL((blk_tri_kernel<float, 3, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 4: hipLaunchKernelGGL((blk_tri_kernel<float, 4, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 5: hipLaunchKernelGGL((blk_tri_kernel<float, 5, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 6: hipLaunchKernelGGL((blk_tri_kernel<float, 6, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 7: hipLaunchKernelGGL((blk_tri_kernel<float, 7, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 8: hipLaunchKernelGGL((blk_tri_kernel<float, 8, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 9: hipLaunchKernelGGL((blk_tri_kernel<float, 9, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 10: hipLaunchKernelGGL((blk_tri_kernel<float, 10, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 11: hipLaunchKernelGGL((blk_tri_kernel<float, 11, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 12: hipLaunchKernelGGL((blk_tri_kernel<float, 12, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 13: hipLaunchKernelGGL((blk_tri_kernel<float, 13, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 14: hipLaunchKernelGGL((blk_tri_kernel<float, 14, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 15: hipLaunchKernelGGL((blk_tri_kernel<float, 15, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 16: hipLaunchKernelGGL((blk_tri_kernel<float, 16, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    default: return false;
    }
}

bool launch_zupd(int m, const ZupdArgsT<float> &a, hipStream_t st)
{
    if (a.lo <= a.r0) return true;
    if (!zupd_args_ok(m, a)) return false;
    const int w = blk_cols(m, a.nr != 0);
    const dim3 grid((unsigned)((a.ncols / zupd_bn(w)) * ((a.lo - a.r0 + 127) / 128)));
    switch (w) {
    case 2: hipLaunchKernelGGL((zupd32_kernel<2>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 4: hipLaunchKernelGGL((zupd32_kernel<4>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 8: hipLaunchKernelGGL((zupd32_kernel<8>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 16: hipLaunchKernelGGL((zupd32_kernel<16>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 24: hipLaunchKernelGGL((zupd32_kernel<24>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 32: hipLaunchKernelGGL((zupd32_kernel<32>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 48: hipLaunchKernelGGL((zupd32_kernel<48>), grid, dim3(256), kZupd32Lds, st, a); return true;
    case 64: hipLaunchKernelGGL((zupd32_kernel<64>), grid, dim3(256), kZupd32Lds, st, a); return true;
    default: return false;
    }
}


}  // namespace shs
