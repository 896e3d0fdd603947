// inst_stream.hpp -- launch wrappers and registration for the fused kernels.
#pragma once

#include "registry.hpp"
#include "seg1d_kernel.hpp"
#include "stream_kernel.hpp"
#include "variants.hpp"

namespace stn {

template <typename S> constexpr int storage_dtype() {
    if constexpr (std::is_same<S, double>::value) return kF64;
    if constexpr (std::is_same<S, float>::value) return kF32;
    if constexpr (std::is_same<S, bf16_t>::value) return kBF16;
    return kF16;
}

template <int DIM> constexpr int variant_id(int vx, int nw, int rw) {
    constexpr int n = DIM == 3 ? kNumV3 : (DIM == 2 ? kNumV2 : kNumV1);
    for (int i = 1; i <= n; ++i) {
        const VariantShape v = variant_of<DIM>(i);
        if (v.vx == vx && v.nw == nw && (DIM != 3 || v.rw == rw)) return i;
    }
    return 0;
}

template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW>
hipError_t launch_stream(const SweepLaunch &L, hipStream_t st) {
    using C = typename ComputeOf<S>::type;
    const Geometry g = stream_geometry(DIM, R, K, VariantShape{VX, NW, RW}, L.n0, L.n1, L.n2, L.chunk);
    if (!g.ok) return hipErrorInvalidValue;
    StreamArgs<C> a;
    a.src = L.src;
    a.dst = L.dst;
    a.n0 = L.n0;
    a.n1 = L.n1;
    a.n2 = L.n2;
    a.tiles_x = g.tiles_x;
    a.tiles_y = g.tiles_y;
    a.chunks = g.chunks;
    a.chunk = g.chunk;
    a.out_x = g.out_x;
    a.out_y = g.out_y;
    a.halo_x = g.halo_x;
    a.bc = L.bc;
    a.nblocks = g.nblocks;
    constexpr int W = 2 * R + 1;
    constexpr int nd = DIM == 3 ? W * W * W : W * W;
    static_assert(nd <= kMaxDense, "dense table too large");
    for (int i = 0; i < kMaxDense; ++i) a.coef[i] = i < nd ? (C)L.dense[i] : C(0);
    hipLaunchKernelGGL((stream_kernel<S, DIM, R, BOX, K, VX, NW, RW>), dim3(g.nblocks),
                       dim3(g.threads), 0, st, a);
    return hipGetLastError();
}

// workgroups of one streaming kernel a compute unit holds (queried once)
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW> int occupancy_stream() {
    static int per = -1;
    if (per < 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &v, reinterpret_cast<const void *>(&stream_kernel<S, DIM, R, BOX, K, VX, NW, RW>), 64 * NW, 0) !=
            hipSuccess)
            v = 0;
        per = v;
    }
    return per;
}

template <typename S, int R, int K, int VX, int NW>
hipError_t launch_seg1d(const SweepLaunch &L, hipStream_t st) {
    using C = typename ComputeOf<S>::type;
    const Geometry g = seg1d_geometry(R, K, VariantShape{VX, NW, 1}, L.n2);
    if (!g.ok) return hipErrorInvalidValue;
    Seg1DArgs<C> a;
    a.src = L.src;
    a.dst = L.dst;
    a.n = L.n2;
    a.tiles = g.tiles_x;
    a.out_x = g.out_x;
    a.halo_x = g.halo_x;
    a.bc = L.bc;
    a.nblocks = g.nblocks;
    for (int i = 0; i < 9; ++i) a.coef[i] = i < 2 * R + 1 ? (C)L.dense[i] : C(0);
    hipLaunchKernelGGL((seg1d_kernel<S, R, K, VX, NW>), dim3(g.nblocks), dim3(g.threads), 0, st, a);
    return hipGetLastError();
}

template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int K>
struct StreamReg {
    StreamReg() {
        constexpr int vid = variant_id<DIM>(VX, NW, RW);
        static_assert(vid > 0, "shape is not a listed variant");
        register_launcher(KernelKey{storage_dtype<S>(), DIM, R, BOX ? 1 : 0, vid, K},
                          &launch_stream<S, DIM, R, BOX, K, VX, NW, RW>,
                          &occupancy_stream<S, DIM, R, BOX, K, VX, NW, RW>);
    }
};

template <typename S, int R, int VX, int NW, int K> struct Seg1DReg {
    Seg1DReg() {
        constexpr int vid = variant_id<1>(VX, NW, 1);
        static_assert(vid > 0, "shape is not a listed variant");
        // in 1D the star and the box are the same offset set
        register_launcher(KernelKey{storage_dtype<S>(), 1, R, 0, vid, K}, &launch_seg1d<S, R, K, VX, NW>);
        register_launcher(KernelKey{storage_dtype<S>(), 1, R, 1, vid, K}, &launch_seg1d<S, R, K, VX, NW>);
    }
};

// register K = 1..KMAX of one (type, stencil, variant)
template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int... Ks>
struct StreamRegs {
    StreamRegs() { (void)std::initializer_list<int>{(StreamReg<S, DIM, R, BOX, VX, NW, RW, Ks>(), 0)...}; }
};
template <typename S, int R, int VX, int NW, int... Ks> struct Seg1DRegs {
    Seg1DRegs() { (void)std::initializer_list<int>{(Seg1DReg<S, R, VX, NW, Ks>(), 0)...}; }
};

}  // namespace stn
