// Instances of the blocked FP64 tile kernel with a dense right-hand side
// (transposed systems), m = 1 .. 16.
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool launch_blk_tri_dense(int m, const BlkTriArgsT<double> &a, hipStream_t st)
{
    switch (m) {
    case 1: hipLaunchKernelGGL((blk_tri_kernel<double, 1, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 2: hipLaunchKernelGGL((blk_tri_kernel<double, 2, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 3: hipLaunchKernelGGL((blk_tri_kernel<double, 3, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 4: hipLaunchKernelGGL((blk_tri_kernel<double, 4, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 5: hipLaunchKernelGGL((blk_tri_kernel<double, 5, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 6: hipLaunchKernelGGL((blk_tri_kernel<double, 6, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 7: hipLaunchKernelGGL((blk_tri_kernel<double, 7, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 8: hipLaunchKernelGGL((blk_tri_kernel<double, 8, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 9: hipLaunchKernelGGL((blk_tri_kernel<double, 9, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 10: hipLaunchKernelGGL((blk_tri_kernel<double, 10, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 11: hipLaunchKernelGGL((blk_tri_kernel<double, 11, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 12: hipLaunchKernelGGL((blk_tri_kernel<double, 12, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 13: hipLaunchKernelGGL((blk_tri_kernel<double, 13, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 14: hipLaunchKernelGGL((blk_tri_kernel<double, 14, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 15: hipLaunchKernelGGL((blk_tri_kernel<double, 15, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    case 16: hipLaunchKernelGGL((blk_tri_kernel<double, 16, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
    default: return false;
    }
}

}  // namespace shs
