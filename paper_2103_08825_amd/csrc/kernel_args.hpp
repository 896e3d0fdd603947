// kernel_args.hpp -- argument blocks passed by value to the stencil kernels.
#pragma once

#include <stdint.h>

namespace stn {

constexpr int kMaxDense = 125;  // (2R+1)^DIM for R <= 2 in 3D, R <= 5 in 2D

// Fused streaming sweep (2D and 3D).  Axis 0 is streamed; for 2D n1 == 1.
template <typename C> struct StreamArgs {
    const void *src;
    void *dst;
    int64_t n0, n1, n2;
    int tiles_x, tiles_y;  // output tiles along x and y (tiles_y == 1 in 2D)
    int chunks, chunk;     // chunks of `chunk` output planes along axis 0
    int out_x, out_y;      // output tile extents
    int halo_x;            // x halo of the widened tile (>= K*R, multiple of VX)
    int bc;                // 0 zero halo, 1 periodic
    int nblocks;           // launched workgroups
    // tessellated stages only: y tiles of tile_h rows (the last starts at
    // last_start), ncut cuts, slope buffer in compute precision
    int tile_h, last_start, ncut;
    void *slope;           // tessellated: slope buffer; in place: side buffer
    // in place only: side-buffer elements per band block and per whole-plane
    // block, offset of the whole-plane blocks, x tiles per workgroup
    int64_t side_band, side_zplane, side_z0;
    int side_nw;
    // fused adjoint only: the forward state each level pairs with (level j:
    // ustate[j-1]) and the FP64 gradient partials, one row of npts per wave
    const void *ustate[8];
    double *gpart;
    int npts;
    C coef[kMaxDense];     // dense weight table, [dz][dy][dx] in 3D, [dz][dx] in 2D
};

// Fused 1D sweep: each wave advances one widened segment K steps in registers.
template <typename C> struct Seg1DArgs {
    const void *src;
    void *dst;
    int64_t n;
    int tiles, out_x, halo_x, bc, nblocks;
    C coef[9];             // dense, index dx + R (R <= 4)
};

// Reference sweep: one output point per thread, any d <= 3 and r <= 4,
// neighbours read straight from memory.  Grids are padded to three axes.
template <typename C> struct GenericArgs {
    const void *src;
    void *dst;
    int64_t n0, n1, n2;
    int npts, bc;
    const int *off;        // device, npts*3 ints (axis 0..2 of the padded grid)
    const C *coef;         // device, npts weights in canonical order
};

}  // namespace stn
