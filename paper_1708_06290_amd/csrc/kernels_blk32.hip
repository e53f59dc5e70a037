// Instances of the blocked FP32 tile kernel (the mixed-precision sweep) for
// m = 1 .. 16 with the structured right-hand side and m = 1 .. 8 with a dense
// one (the correction solves).
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool launch_blk_tri(int m, bool dense, const BlkTriArgsT<float> &a, hipStream_t st)
{
    bool ok = false;
    if (!dense) {
        SHS_DISPATCH_M(m, {
            hipLaunchKernelGGL((blk_tri_kernel<float, MM, false>), dim3(a.count), dim3(kWave), 0, st, a);
            ok = true;
        });
    } else {
        switch (m) {
        case 1: hipLaunchKernelGGL((blk_tri_kernel<float, 1, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 2: hipLaunchKernelGGL((blk_tri_kernel<float, 2, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 3: hipLaunchKernelGGL((blk_tri_kernel<float, 3, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 4: hipLaunchKernelGGL((blk_tri_kernel<float, 4, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 5: hipLaunchKernelGGL((blk_tri_kernel<float, 5, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 6: hipLaunchKernelGGL((blk_tri_kernel<float, 6, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 7: hipLaunchKernelGGL((blk_tri_kernel<float, 7, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        case 8: hipLaunchKernelGGL((blk_tri_kernel<float, 8, true>), dim3(a.count), dim3(kWave), 0, st, a); return true;
        default: return false;
        }
    }
    return ok;
}

}  // namespace shs
