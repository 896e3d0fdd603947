// Persistent batched-sweep kernel, f64 storage.
#include "batched_kernel.hpp"

namespace stn {

hipError_t launch_batched_f64(const BatchArgs &a, int wgs, hipStream_t st) {
    hipLaunchKernelGGL(batched_kernel<double>, dim3(wgs), dim3(64 * kBatchNW), 0, st, a);
    return hipGetLastError();
}

const void *batched_kernel_f64() { return reinterpret_cast<const void *>(&batched_kernel<double>); }

}  // namespace stn
