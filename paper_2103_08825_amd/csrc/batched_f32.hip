// Persistent batched-sweep kernel, f32 storage.
#include "batched_kernel.hpp"

namespace stn {

hipError_t launch_batched_f32(const BatchArgs &a, int wgs, hipStream_t st) {
    hipLaunchKernelGGL(batched_kernel<float>, dim3(wgs), dim3(64 * kBatchNW), 0, st, a);
    return hipGetLastError();
}

const void *batched_kernel_f32() { return reinterpret_cast<const void *>(&batched_kernel<float>); }

}  // namespace stn
