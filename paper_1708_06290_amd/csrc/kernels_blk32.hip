// Instances of the blocked FP32 tile kernel (the mixed-precision sweep) for
// m = 1 .. 16 with the structured right-hand side (the dense one and the FP32
// update GEMM: kernels_blk32_dense.hip).
#include "blocked.hpp"
#include "kernels.hpp"

namespace shs {

bool launch_blk_tri(int m, bool dense, const BlkTriArgsT<float> &a, hipStream_t st)
{
    if (dense) return launch_blk_tri_dense(m, a, st);
    bool ok = false;
    SHS_DISPATCH_M(m, {
        hipLaunchKernelGGL((blk_tri_kernel<float, MM, false>), dim3(a.count), dim3(kWave), 0, st, a);
        ok = true;
    });
    return ok;
}

}  // namespace shs
