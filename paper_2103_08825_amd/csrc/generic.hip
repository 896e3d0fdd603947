// generic.hip -- launcher of the reference one-step sweep kernel.
#include "generic_kernel.hpp"
#include "launch.hpp"

namespace stn {

template <typename S>
static hipError_t launch_generic_t(const void *src, void *dst, int64_t n0, int64_t n1, int64_t n2,
                                   int npts, int bc, const int *d_off, const void *d_coef,
                                   hipStream_t st) {
    using C = typename ComputeOf<S>::type;
    GenericArgs<C> a;
    a.src = src;
    a.dst = dst;
    a.n0 = n0;
    a.n1 = n1;
    a.n2 = n2;
    a.npts = npts;
    a.bc = bc;
    a.off = d_off;
    a.coef = static_cast<const C *>(d_coef);
    const int64_t total = n0 * n1 * n2;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;  // grid-stride beyond this
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(generic_kernel<S>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_generic(int dtype, const void *src, void *dst, int64_t n0, int64_t n1,
                          int64_t n2, int npts, int bc, const int *d_off, const void *d_coef,
                          hipStream_t st) {
    switch (dtype) {
    case kF64: return launch_generic_t<double>(src, dst, n0, n1, n2, npts, bc, d_off, d_coef, st);
    case kF32: return launch_generic_t<float>(src, dst, n0, n1, n2, npts, bc, d_off, d_coef, st);
    case kBF16: return launch_generic_t<bf16_t>(src, dst, n0, n1, n2, npts, bc, d_off, d_coef, st);
    case kF16: return launch_generic_t<_Float16>(src, dst, n0, n1, n2, npts, bc, d_off, d_coef, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace stn
