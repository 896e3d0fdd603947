// reduce.hip -- FP64 reductions over a stored field: sum, sum of squares,
// max |u|, and the same against a reference field.  Fixed partial layout
// (kReduceBlocks x 256 threads, grid-stride order, fixed tree order), so the
// result is deterministic for a given element count.
#include <mutex>

#include "device_common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stn {

constexpr int kReduceBlocks = 2048;  // partial slots (a launch uses <= this many)
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

struct Acc6 {
    double s, s2, mx, d2, dmx, rmx;
};

__device__ __forceinline__ void acc_add(Acc6 &a, double x, const double *y) {
    a.s += x;
    a.s2 += x * x;
    a.mx = fmax(a.mx, fabs(x));
    if (y) {
        const double d = x - *y;
        a.d2 += d * d;
        a.dmx = fmax(a.dmx, fabs(d));
        a.rmx = fmax(a.rmx, fabs(*y));
    }
}

// block-wide fold of the six values in a fixed order; result valid in thread 0
__device__ __forceinline__ Acc6 block_fold(Acc6 a) {
    __shared__ double sh[6][kReduceThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    a.s = wave_sum(a.s);
    a.s2 = wave_sum(a.s2);
    a.mx = wave_max(a.mx);
    a.d2 = wave_sum(a.d2);
    a.dmx = wave_max(a.dmx);
    a.rmx = wave_max(a.rmx);
    if (lane == 0) {
        sh[0][w] = a.s;
        sh[1][w] = a.s2;
        sh[2][w] = a.mx;
        sh[3][w] = a.d2;
        sh[4][w] = a.dmx;
        sh[5][w] = a.rmx;
    }
    __syncthreads();
    Acc6 r{sh[0][0], sh[1][0], sh[2][0], sh[3][0], sh[4][0], sh[5][0]};
    for (int k = 1; k < kReduceThreads / 64; ++k) {
        r.s += sh[0][k];
        r.s2 += sh[1][k];
        r.mx = fmax(r.mx, sh[2][k]);
        r.d2 += sh[3][k];
        r.dmx = fmax(r.dmx, sh[4][k]);
        r.rmx = fmax(r.rmx, sh[5][k]);
    }
    return r;
}

// Each thread folds groups of G consecutive elements, grid-stride; the launch
// shape depends only on n, so the summation order is fixed for a given n
// (G = 4 when both pointers allow vector loads, else 1).
template <typename S, int G>
__global__ void __launch_bounds__(kReduceThreads)
    reduce_partials(const S *__restrict__ u, const S *__restrict__ ref, int64_t n, double *part) {
    Acc6 a{0, 0, 0, 0, 0, 0};
    const int64_t ngroups = n / G;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
        const VecS<S, G> tu = *reinterpret_cast<const VecS<S, G> *>(u + G * g);
        if (ref) {
            const VecS<S, G> tr = *reinterpret_cast<const VecS<S, G> *>(ref + G * g);
#pragma unroll
            for (int v = 0; v < G; ++v) {
                const double y = (double)to_compute(tr.v[v]);
                acc_add(a, (double)to_compute(tu.v[v]), &y);
            }
        } else {
#pragma unroll
            for (int v = 0; v < G; ++v) acc_add(a, (double)to_compute(tu.v[v]), nullptr);
        }
    }
    // tail of n mod G elements: block 0
    if (blockIdx.x == 0 && threadIdx.x < (int)(n - G * ngroups)) {
        const int64_t i = G * ngroups + threadIdx.x;
        const double y = ref ? (double)to_compute(ref[i]) : 0.0;
        acc_add(a, (double)to_compute(u[i]), ref ? &y : nullptr);
    }
    const Acc6 r = block_fold(a);
    if (threadIdx.x == 0) {
        double *p = part + (int64_t)blockIdx.x * 6;
        p[0] = r.s;
        p[1] = r.s2;
        p[2] = r.mx;
        p[3] = r.d2;
        p[4] = r.dmx;
        p[5] = r.rmx;
    }
}

__global__ void __launch_bounds__(kReduceThreads) reduce_final(const double *__restrict__ part, int nb, double *out) {
    Acc6 a{0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kReduceThreads) {
        const double *p = part + (int64_t)b * 6;
        a.s += p[0];
        a.s2 += p[1];
        a.mx = fmax(a.mx, p[2]);
        a.d2 += p[3];
        a.dmx = fmax(a.dmx, p[4]);
        a.rmx = fmax(a.rmx, p[5]);
    }
    const Acc6 r = block_fold(a);
    if (threadIdx.x == 0) {
        out[0] = r.s;
        out[1] = r.s2;
        out[2] = r.mx;
        out[3] = r.d2;
        out[4] = r.dmx;
        out[5] = r.rmx;
    }
}

template <typename S>
static hipError_t launch_reduce_t(const void *u, const void *ref, int64_t n, double *part, double *out,
                                  hipStream_t st) {
    // enough workgroups to stream at full bandwidth, fewer for small n
    int64_t nb = (n / 4 + kReduceThreads * 8 - 1) / (kReduceThreads * 8);
    if (nb < 1) nb = 1;
    if (nb > kReduceBlocks) nb = kReduceBlocks;
    const uintptr_t al = 4 * sizeof(S);
    if ((uintptr_t)u % al == 0 && (uintptr_t)ref % al == 0)
        hipLaunchKernelGGL((reduce_partials<S, 4>), dim3((unsigned)nb), dim3(kReduceThreads), 0, st,
                           static_cast<const S *>(u), static_cast<const S *>(ref), n, part);
    else
        hipLaunchKernelGGL((reduce_partials<S, 1>), dim3((unsigned)nb), dim3(kReduceThreads), 0, st,
                           static_cast<const S *>(u), static_cast<const S *>(ref), n, part);
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kReduceThreads), 0, st, (const double *)part, (int)nb, out);
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

// ---------------------------------------------------------------------------
// Allocation-free variant of the reduction: the partial rows live in a fixed
// device array instead of a stream-ordered allocation.  A launch never uses
// more than kReduceBlocks rows, whatever n is, so the array has a fixed size.
namespace stn {

constexpr int kScratchDoubles = kReduceBlocks * 6;  // 96 KiB
constexpr int kMaxDevices = 64;

// In host code this name is only a stand-in for the symbol: the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// The current device's copy of `scratch` (looked up on the first call on each
// device, with that device current).
static int scratch_for_current_device(double **out) {
    int dev = 0;
    STN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(STENCIL_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(STENCIL_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return STENCIL_OK;
}

}  // namespace stn

extern "C" int stencil_reduce_noalloc(int dtype, const void *d_u, const void *d_ref, int64_t n,
                                      double *d_out, void *stream) {
    using namespace stn;
    clear_error();
    if (elem_bytes(dtype) == 0) return fail(STENCIL_E_INVALID, "unknown dtype %d", dtype);
    if (n < 0) return fail(STENCIL_E_INVALID, "n must be >= 0");
    if (!d_out || (!d_u && n > 0)) return fail(STENCIL_E_INVALID, "NULL pointer");
    if (reduce_partials_bytes() > (int)sizeof(scratch))
        return fail(STENCIL_E_INVALID, "partial rows need %d bytes, the fixed scratch holds %d",
                    reduce_partials_bytes(), (int)sizeof(scratch));
    double *part = nullptr;
    const int rc = scratch_for_current_device(&part);
    if (rc != STENCIL_OK) return rc;
    // every partial row the final fold reads is written by this call's first
    // kernel, so nothing needs clearing
    const hipError_t e = launch_reduce(dtype, d_u, d_ref, n, part, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "reduction launch: %s", hipGetErrorString(e));
    return STENCIL_OK;
}
