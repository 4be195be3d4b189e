// The batch sweep kernel (every block size in one kernel) and its launcher,
// in a translation unit of their own.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace bilu {
namespace launch {

bool batch_sweep(bool fp32, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::BatchSweepArgs& a)
{
    if (fuse) {
        if (fp32) hipLaunchKernelGGL((dev::k_sweep_batch<float, true>), dim3(blocks), dim3(64), lds, s, a);
        else hipLaunchKernelGGL((dev::k_sweep_batch<double, true>), dim3(blocks), dim3(64), lds, s, a);
    } else {
        if (fp32) hipLaunchKernelGGL((dev::k_sweep_batch<float, false>), dim3(blocks), dim3(64), lds, s, a);
        else hipLaunchKernelGGL((dev::k_sweep_batch<double, false>), dim3(blocks), dim3(64), lds, s, a);
    }
    return true;
}

}  // namespace launch
}  // namespace bilu
