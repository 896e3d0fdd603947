// seg1d_kernel.hpp -- fused multi-step sweep for 1D grids.
//
// Each 64-wide wave owns one output segment widened by a halo of K*R points
// (VX consecutive points per lane), loads it once, advances it K steps in
// registers -- neighbours from the lane's own registers or from the adjacent
// lane through whole-wave DPP shifts -- and stores the segment's interior
// (Section 3.3: K steps per load/store instead of one).  The halo shrinks by
// R per step and is recomputed by the neighbouring segment's wave.
#pragma once

#include "device_common.hpp"
#include "kernel_args.hpp"

namespace stn {

template <int DX, int V, int VX, typename C> __device__ __forceinline__ C xval1d(const C (&row)[VX]) {
    constexpr int t = V + DX;
    constexpr int s = floordiv(t, VX);
    constexpr int m = t - s * VX;
    return lane_shift<s>(row[m]);
}

template <typename S, int R, int K, int VX, int NW>
__global__ void __launch_bounds__(64 * NW) seg1d_kernel(const Seg1DArgs<typename ComputeOf<S>::type> a) {
    using C = typename ComputeOf<S>::type;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int tile = xcd_remap(blockIdx.x, a.nblocks) * NW + wv;
    if (tile >= a.tiles) return;
    const S *__restrict__ src = static_cast<const S *>(a.src);
    S *__restrict__ dst = static_cast<S *>(a.dst);
    const bool periodic = (a.bc == 1);
    const int64_t n = a.n;

    const int64_t x_out0 = (int64_t)tile * a.out_x;
    const int64_t x_hi = (x_out0 + a.out_x < n) ? x_out0 + a.out_x : n;
    const int64_t x_lane = x_out0 - a.halo_x + (int64_t)lane * VX;
    bool x_in[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) x_in[v] = (x_lane + v >= 0) && (x_lane + v < n);

    C u[VX];
    if (x_lane >= 0 && x_lane + VX <= n) {
        const VecS<S, VX> t = *reinterpret_cast<const VecS<S, VX> *>(src + x_lane);
#pragma unroll
        for (int v = 0; v < VX; ++v) u[v] = to_compute(t.v[v]);
    } else {
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const int64_t x = x_lane + v;
            if (periodic)
                u[v] = to_compute(src[wrap_index(x, n)]);
            else
                u[v] = x_in[v] ? to_compute(src[x]) : C(0);
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        C nu[VX];
        static_for<0, VX>([&](auto V_) {
            constexpr int V = decltype(V_)::value;
            C t = C(0);
            static_for<-R, R + 1>([&](auto DX_) {
                constexpr int DX = decltype(DX_)::value;
                t = fma_c(a.coef[DX + R], xval1d<DX, V, VX>(u), t);
            });
            nu[V] = t;
        });
#pragma unroll
        for (int v = 0; v < VX; ++v) u[v] = (periodic || x_in[v]) ? nu[v] : C(0);
    }

    if (x_lane >= x_out0 && x_lane + VX <= x_hi) {
        VecS<S, VX> t;
#pragma unroll
        for (int v = 0; v < VX; ++v) t.v[v] = from_compute<S>(u[v]);
        *reinterpret_cast<VecS<S, VX> *>(dst + x_lane) = t;
    } else {
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const int64_t x = x_lane + v;
            if (x >= x_out0 && x < x_hi) dst[x] = from_compute<S>(u[v]);
        }
    }
}

}  // namespace stn
