// registry.hpp -- lookup of the compiled fused kernels.
//
// Each instantiation unit registers its launchers from a static initialiser
// when the library is loaded; plans look them up by
// (dtype, dim, radius, box, variant, k).
#pragma once

#include "launch.hpp"

namespace stn {

struct KernelKey {
    int dtype, dim, r, box, variant, k;
    int mode;  // 0: fused (overlapped) pass; 1: tessellated pass (both stages); 2: in-place pass;
               // 3: fused adjoint pass (mirrored steps with the coefficient gradient);
               // 4: fused pass storing every intermediate level
};

// workgroups of one kernel that a compute unit holds at once (0 if unknown)
using OccupancyFn = int (*)();

void register_launcher(const KernelKey &key, SweepLauncher fn, OccupancyFn occ = nullptr);
SweepLauncher find_launcher(const KernelKey &key);
// workgroups of the kernel behind `key` the whole device holds at once (0 if unknown)
int resident_blocks(const KernelKey &key);
// largest k registered for (dtype, dim, r, box, variant, mode); 0 if none
int registered_max_k(int dtype, int dim, int r, int box, int variant, int mode = 0);
// every registered key
int registered_keys(KernelKey *out, int cap);

template <typename S> constexpr int dtype_of();
template <> constexpr int dtype_of<double>() { return kF64; }
template <> constexpr int dtype_of<float>() { return kF32; }

}  // namespace stn
