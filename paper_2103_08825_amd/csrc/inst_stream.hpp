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

// One in-place pass (src == dst): the fused kernel storing band points to the
// side buffer L.aux, then the fix-up copying them into the field.
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW>
hipError_t launch_inplace(const SweepLaunch &L, hipStream_t st) {
    using C = typename ComputeOf<S>::type;
    const VariantShape vs{VX, NW, RW};
    const Geometry g = stream_geometry(DIM, R, K, vs, L.n0, L.n1, L.n2, L.chunk);
    const InplaceSide side = inplace_side(DIM, R, K, vs, L.n0, L.n1, L.n2, L.chunk);
    if (!g.ok || !side.ok || !L.aux || L.src != L.dst) return hipErrorInvalidValue;
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
    a.slope = L.aux;
    a.side_band = side.band;
    a.side_zplane = side.zplane;
    a.side_z0 = side.z0;
    a.side_nw = DIM == 3 ? 1 : NW;
    constexpr int W = 2 * R + 1;
    constexpr int nd = DIM == 3 ? W * W * W : W * W;
    for (int i = 0; i < kMaxDense; ++i) a.coef[i] = i < nd ? (C)L.dense[i] : C(0);
    hipLaunchKernelGGL((stream_kernel<S, DIM, R, BOX, K, VX, NW, RW, kInPlace>), dim3(g.nblocks), dim3(g.threads), 0,
                       st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nfix = (int64_t)g.nblocks * kFixupParts;
    if (nfix > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((inplace_fixup<S, DIM, R, K>), dim3((unsigned)nfix), dim3(256), 0, st, a);
    return hipGetLastError();
}

// One fused adjoint launch: K mirrored steps with the gradient folded in
// (L.dense holds the mirrored weights; L.ustate[j-1] the forward state of
// level j; L.gpart the partial rows).
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW>
hipError_t launch_adjoint(const SweepLaunch &L, hipStream_t st) {
    using C = typename ComputeOf<S>::type;
    const Geometry g = stream_geometry(DIM, R, K, VariantShape{VX, NW, RW}, L.n0, L.n1, L.n2, L.chunk);
    if (!g.ok || !L.gpart) return hipErrorInvalidValue;
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
    for (int j = 0; j < 8; ++j) a.ustate[j] = j < K ? L.ustate[j] : nullptr;
    a.gpart = L.gpart;
    constexpr int W = 2 * R + 1;
    constexpr int nd = DIM == 3 ? W * W * W : W * W;
    a.npts = num_terms<DIM, R, BOX>();
    for (int i = 0; i < kMaxDense; ++i) a.coef[i] = i < nd ? (C)L.dense[i] : C(0);
    hipLaunchKernelGGL((stream_kernel<S, DIM, R, BOX, K, VX, NW, RW, kAdjoint>), dim3(g.nblocks), dim3(g.threads),
                       0, st, a);
    return hipGetLastError();
}

// One fused pass of K steps that also stores every intermediate level (level
// j < K to L.ustate[j-1], level K to L.dst).
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW>
hipError_t launch_levels(const SweepLaunch &L, hipStream_t st) {
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
    for (int j = 0; j < 8; ++j) a.ustate[j] = j < K - 1 ? L.ustate[j] : nullptr;
    constexpr int W = 2 * R + 1;
    constexpr int nd = DIM == 3 ? W * W * W : W * W;
    for (int i = 0; i < kMaxDense; ++i) a.coef[i] = i < nd ? (C)L.dense[i] : C(0);
    hipLaunchKernelGGL((stream_kernel<S, DIM, R, BOX, K, VX, NW, RW, kLevels>), dim3(g.nblocks), dim3(g.threads),
                       0, st, a);
    return hipGetLastError();
}

// workgroups of one streaming kernel a compute unit holds (queried once)
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW, int MODE = kOverlapped>
int occupancy_stream() {
    static int per = -1;
    if (per < 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &v, reinterpret_cast<const void *>(&stream_kernel<S, DIM, R, BOX, K, VX, NW, RW, MODE>), 64 * NW, 0) !=
            hipSuccess)
            v = 0;
        per = v;
    }
    return per;
}

// One tessellated pass of K steps on a 3D grid: stage A on tiles of NWA*RWA
// rows, then stage B on frames of NWB*RWA rows around the cuts (both on `st`).
template <typename S, int R, bool BOX, int K, int VX, int NWA, int RWA, int NWB>
hipError_t launch_tess(const SweepLaunch &L, hipStream_t st) {
    using C = typename ComputeOf<S>::type;
    static_assert(NWB * RWA >= 2 * (K + 1) * R, "stage-B frame too short");
    const Geometry g = stream_geometry(3, R, K, VariantShape{VX, NWA, RWA}, L.n0, L.n1, L.n2, L.chunk);
    const TessTiling t = tess_tiling(R, K, NWA * RWA, L.n1, L.bc);
    if (!g.ok || !t.ok || (K >= 2 && !L.aux)) return hipErrorInvalidValue;
    StreamArgs<C> a;
    a.src = L.src;
    a.dst = L.dst;
    a.n0 = L.n0;
    a.n1 = L.n1;
    a.n2 = L.n2;
    a.tiles_x = g.tiles_x;
    a.tiles_y = t.tiles_y;
    a.chunks = g.chunks;
    a.chunk = g.chunk;
    a.out_x = g.out_x;
    a.out_y = 0;
    a.halo_x = g.halo_x;
    a.bc = L.bc;
    a.tile_h = t.tile_h;
    a.last_start = t.last_start;
    a.ncut = t.ncut;
    a.slope = L.aux;
    for (int i = 0; i < kMaxDense; ++i) a.coef[i] = i < (2 * R + 1) * (2 * R + 1) * (2 * R + 1) ? (C)L.dense[i] : C(0);
    const int64_t na = (int64_t)g.tiles_x * t.tiles_y * g.chunks;
    const int64_t nb = (int64_t)g.tiles_x * t.ncut * g.chunks;
    if (na > 0x7fffffff || nb > 0x7fffffff) return hipErrorInvalidValue;
    a.nblocks = (int)na;
    hipLaunchKernelGGL((stream_kernel<S, 3, R, BOX, K, VX, NWA, RWA, kTessA>), dim3(a.nblocks), dim3(64 * NWA),
                       0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.nblocks = (int)nb;
    hipLaunchKernelGGL((stream_kernel<S, 3, R, BOX, K, VX, NWB, RWA, kTessB>), dim3(a.nblocks), dim3(64 * NWB),
                       0, st, a);
    return hipGetLastError();
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

template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int K> struct InplaceReg {
    InplaceReg() {
        constexpr int vid = variant_id<DIM>(VX, NW, RW);
        static_assert(vid > 0, "shape is not a listed variant");
        register_launcher(KernelKey{storage_dtype<S>(), DIM, R, BOX ? 1 : 0, vid, K, 2},
                          &launch_inplace<S, DIM, R, BOX, K, VX, NW, RW>);
    }
};
// register the in-place pass for K = Ks...
template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int... Ks> struct InplaceRegs {
    InplaceRegs() { (void)std::initializer_list<int>{(InplaceReg<S, DIM, R, BOX, VX, NW, RW, Ks>(), 0)...}; }
};

template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int K> struct AdjointReg {
    AdjointReg() {
        constexpr int vid = variant_id<DIM>(VX, NW, RW);
        static_assert(vid > 0, "shape is not a listed variant");
        register_launcher(KernelKey{storage_dtype<S>(), DIM, R, BOX ? 1 : 0, vid, K, 3},
                          &launch_adjoint<S, DIM, R, BOX, K, VX, NW, RW>,
                          &occupancy_stream<S, DIM, R, BOX, K, VX, NW, RW, kAdjoint>);
    }
};
template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int K> struct LevelsReg {
    LevelsReg() {
        constexpr int vid = variant_id<DIM>(VX, NW, RW);
        static_assert(vid > 0, "shape is not a listed variant");
        register_launcher(KernelKey{storage_dtype<S>(), DIM, R, BOX ? 1 : 0, vid, K, 4},
                          &launch_levels<S, DIM, R, BOX, K, VX, NW, RW>,
                          &occupancy_stream<S, DIM, R, BOX, K, VX, NW, RW, kLevels>);
    }
};
// register the level-storing pass for K = Ks...
template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int... Ks> struct LevelsRegs {
    LevelsRegs() { (void)std::initializer_list<int>{(LevelsReg<S, DIM, R, BOX, VX, NW, RW, Ks>(), 0)...}; }
};
// register the fused adjoint pass for K = Ks...
template <typename S, int DIM, int R, bool BOX, int VX, int NW, int RW, int... Ks> struct AdjointRegs {
    AdjointRegs() { (void)std::initializer_list<int>{(AdjointReg<S, DIM, R, BOX, VX, NW, RW, Ks>(), 0)...}; }
};

template <typename S, int R, bool BOX, int VX, int NWA, int RWA, int NWB, int K> struct TessReg {
    TessReg() {
        constexpr int vid = variant_id<3>(VX, NWA, RWA);
        static_assert(vid > 0, "stage-A shape is not a listed variant");
        register_launcher(KernelKey{storage_dtype<S>(), 3, R, BOX ? 1 : 0, vid, K, 1},
                          &launch_tess<S, R, BOX, K, VX, NWA, RWA, NWB>);
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
// register the tessellated pass for K = Ks...
template <typename S, int R, bool BOX, int VX, int NWA, int RWA, int NWB, int... Ks> struct TessRegs {
    TessRegs() { (void)std::initializer_list<int>{(TessReg<S, R, BOX, VX, NWA, RWA, NWB, Ks>(), 0)...}; }
};
template <typename S, int R, int VX, int NW, int... Ks> struct Seg1DRegs {
    Seg1DRegs() { (void)std::initializer_list<int>{(Seg1DReg<S, R, VX, NW, Ks>(), 0)...}; }
};

}  // namespace stn
