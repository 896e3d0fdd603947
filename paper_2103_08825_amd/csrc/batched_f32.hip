// Persistent batched-sweep kernel, f32 storage.
#include "batched_kernel.hpp"

namespace stn {

hipError_t launch_batched_f32(const BatchArgs &a, int rmax, int wgs, hipStream_t st) {
    if (rmax <= 1)
        hipLaunchKernelGGL((batched_kernel<float, 1>), dim3(wgs), dim3(64 * kBatchNW), 0, st, a);
    else
        hipLaunchKernelGGL((batched_kernel<float, 2>), dim3(wgs), dim3(64 * kBatchNW), 0, st, a);
    return hipGetLastError();
}

const void *batched_kernel_f32(int rmax) {
    return rmax <= 1 ? reinterpret_cast<const void *>(&batched_kernel<float, 1>)
                     : reinterpret_cast<const void *>(&batched_kernel<float, 2>);
}

}  // namespace stn
