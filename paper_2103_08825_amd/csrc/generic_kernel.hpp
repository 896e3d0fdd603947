// generic_kernel.hpp -- reference one-step sweep for any d <= 3, r <= 4.
//
// One output point per thread: u_{t+1}[x] = sum_j c_j g(u_t, x + o_j), the
// definition of Section 1 evaluated term by term, every neighbour read from
// memory (caches absorb the reuse).  Used for stencils the fused kernels do
// not cover and as the GPU reference path.
#pragma once

#include "device_common.hpp"
#include "kernel_args.hpp"

namespace stn {

template <typename S>
__global__ void __launch_bounds__(256) generic_kernel(const GenericArgs<typename ComputeOf<S>::type> a) {
    using C = typename ComputeOf<S>::type;
    const S *__restrict__ src = static_cast<const S *>(a.src);
    S *__restrict__ dst = static_cast<S *>(a.dst);
    const int64_t n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int64_t total = n0 * n1 * n2;
    const bool periodic = (a.bc == 1);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x2 = p % n2;
        const int64_t x1 = (p / n2) % n1;
        const int64_t x0 = p / (n1 * n2);
        C acc = C(0);
        for (int j = 0; j < a.npts; ++j) {
            int64_t y0 = x0 + a.off[3 * j], y1 = x1 + a.off[3 * j + 1], y2 = x2 + a.off[3 * j + 2];
            C v;
            const bool inside = (y0 >= 0 && y0 < n0) && (y1 >= 0 && y1 < n1) && (y2 >= 0 && y2 < n2);
            if (inside) {
                v = to_compute(src[(y0 * n1 + y1) * n2 + y2]);
            } else if (periodic) {
                y0 = wrap_index(y0, n0);
                y1 = wrap_index(y1, n1);
                y2 = wrap_index(y2, n2);
                v = to_compute(src[(y0 * n1 + y1) * n2 + y2]);
            } else {
                v = C(0);
            }
            acc = fma_c(a.coef[j], v, acc);
        }
        dst[p] = from_compute<S>(acc);
    }
}

}  // namespace stn
