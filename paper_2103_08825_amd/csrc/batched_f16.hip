// Persistent batched-sweep kernel, f16 storage.
#include "batched_kernel.hpp"

namespace stn {

hipError_t launch_batched_f16(const BatchArgs &a, int wgs, hipStream_t st) {
    hipLaunchKernelGGL(batched_kernel<_Float16>, dim3(wgs), dim3(64 * kBatchNW), 0, st, a);
    return hipGetLastError();
}

const void *batched_kernel_f16() { return reinterpret_cast<const void *>(&batched_kernel<_Float16>); }

}  // namespace stn
