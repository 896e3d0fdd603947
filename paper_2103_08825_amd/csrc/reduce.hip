// reduce.hip -- FP64 reductions over a stored field: sum, sum of squares,
// max |u|, and the same against a reference field.  Fixed partial layout
// (kReduceBlocks x 256 threads, grid-stride order, fixed tree order), so the
// result is deterministic for a given element count.
#include "device_common.hpp"
#include "launch.hpp"

namespace stn {

constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename S>
__global__ void __launch_bounds__(kReduceThreads)
    reduce_partials(const S *__restrict__ u, const S *__restrict__ ref, int64_t n, double *part) {
    double s = 0, s2 = 0, mx = 0, d2 = 0, dmx = 0, rmx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)to_compute(u[i]);
        s += a;
        s2 += a * a;
        mx = fmax(mx, fabs(a));
        if (ref) {
            const double b = (double)to_compute(ref[i]);
            const double d = a - b;
            d2 += d * d;
            dmx = fmax(dmx, fabs(d));
            rmx = fmax(rmx, fabs(b));
        }
    }
    __shared__ double sh[6][kReduceThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    s = wave_sum(s);
    s2 = wave_sum(s2);
    mx = wave_max(mx);
    d2 = wave_sum(d2);
    dmx = wave_max(dmx);
    rmx = wave_max(rmx);
    if (lane == 0) {
        sh[0][w] = s;
        sh[1][w] = s2;
        sh[2][w] = mx;
        sh[3][w] = d2;
        sh[4][w] = dmx;
        sh[5][w] = rmx;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        const bool is_max = (q == 2 || q == 4 || q == 5);
        double acc = sh[q][0];
        for (int k = 1; k < kReduceThreads / 64; ++k) acc = is_max ? fmax(acc, sh[q][k]) : acc + sh[q][k];
        part[(int64_t)blockIdx.x * 6 + q] = acc;
    }
}

__global__ void __launch_bounds__(64) reduce_final(const double *__restrict__ part, int nb, double *out) {
    // one wave: lane q < 6 folds column q over the blocks in block order
    const int q = threadIdx.x;
    if (q < 6) {
        const bool is_max = (q == 2 || q == 4 || q == 5);
        double acc = part[q];
        for (int b = 1; b < nb; ++b) {
            const double v = part[(int64_t)b * 6 + q];
            acc = is_max ? fmax(acc, v) : acc + v;
        }
        out[q] = acc;
    }
}

template <typename S>
static hipError_t launch_reduce_t(const void *u, const void *ref, int64_t n, double *part, double *out,
                                  hipStream_t st) {
    hipLaunchKernelGGL(reduce_partials<S>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                       static_cast<const S *>(u), static_cast<const S *>(ref), n, part);
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(64), 0, st, (const double *)part, kReduceBlocks, out);
    return hipGetLastError();
}

int reduce_partials_bytes() { return kReduceBlocks * 6 * (int)sizeof(double); }

hipError_t launch_reduce(int dtype, const void *u, const void *ref, int64_t n, double *part,
                         double *out, hipStream_t st) {
    switch (dtype) {
    case kF64: return launch_reduce_t<double>(u, ref, n, part, out, st);
    case kF32: return launch_reduce_t<float>(u, ref, n, part, out, st);
    case kBF16: return launch_reduce_t<bf16_t>(u, ref, n, part, out, st);
    case kF16: return launch_reduce_t<_Float16>(u, ref, n, part, out, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace stn
