// Persistent batched-sweep kernel, bf16 storage.
#include "batched_kernel.hpp"

namespace stn {

hipError_t launch_batched_bf16(const BatchArgs &a, int wgs, hipStream_t st) {
    hipLaunchKernelGGL(batched_kernel<bf16_t>, dim3(wgs), dim3(64 * kBatchNW), 0, st, a);
    return hipGetLastError();
}

const void *batched_kernel_bf16() { return reinterpret_cast<const void *>(&batched_kernel<bf16_t>); }

}  // namespace stn
