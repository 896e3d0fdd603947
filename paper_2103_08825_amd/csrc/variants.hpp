// variants.hpp -- the fused kernel shapes compiled into the library.
//
// A variant fixes how a workgroup covers its widened tile: VX columns per
// lane (64*VX columns per wave), NW waves, RW rows per wave (3D only).
// Variant ids start at 1; 0 means "choose".
#pragma once

#include "launch.hpp"

namespace stn {

constexpr int kMaxK3 = 6;   // fused steps per launch compiled for 3D
constexpr int kMaxK2 = 8;   // ... for 2D
constexpr int kMaxK1 = 16;  // ... for 1D

constexpr int kNumV3 = 6;
constexpr VariantShape kV3[kNumV3 + 1] = {{0, 0, 0}, {1, 4, 8}, {1, 8, 8}, {2, 4, 8},
                                          {1, 8, 4}, {1, 16, 4}, {2, 8, 4}};
constexpr int kNumV2 = 2;
constexpr VariantShape kV2[kNumV2 + 1] = {{0, 0, 0}, {1, 4, 1}, {4, 4, 1}};
constexpr int kNumV1 = 2;
constexpr VariantShape kV1[kNumV1 + 1] = {{0, 0, 0}, {1, 4, 1}, {4, 4, 1}};

template <int DIM> constexpr VariantShape variant_of(int i) {
    return DIM == 3 ? kV3[i] : (DIM == 2 ? kV2[i] : kV1[i]);
}

// halo LDS bytes of a 3D variant (0 for 2D and single-wave tiles)
constexpr int halo_lds_bytes(int dim, int r, int k, VariantShape v, int elem) {
    return (dim == 3 && v.nw > 1) ? 2 * k * v.nw * 2 * r * 64 * v.vx * elem : 0;
}

constexpr int kMaxLdsBytes = 64 * 1024;

}  // namespace stn
