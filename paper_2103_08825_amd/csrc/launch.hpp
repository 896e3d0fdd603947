// launch.hpp -- host-side geometry and launch templates for the sweep kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_args.hpp"

namespace stn {

enum Dtype { kF64 = 0, kF32 = 1, kBF16 = 2, kF16 = 3 };

// One fused launch: K steps from src to dst.
struct SweepLaunch {
    const void *src;
    void *dst;
    int64_t n0, n1, n2;  // streamed axis, y axis (1 in 2D), x axis; 1D uses n2 only
    int bc;
    const double *dense; // dense weight table: [dz][dy][dx] (3D), [dz][dx] (2D), [dx] (1D)
    int chunk;           // planes per workgroup along axis 0; 0 = automatic
    void *aux;           // tessellated sweeps: the slope buffer (tess_slope_bytes)
    const void *ustate[8];  // fused adjoint: forward state of each level (level j: [j-1])
    double *gpart;          // fused adjoint: gradient partials (adjoint_part_rows rows of npts)
};

using SweepLauncher = hipError_t (*)(const SweepLaunch &, hipStream_t);

// Kernel shape of a fused variant.
struct VariantShape {
    int vx, nw, rw;
};

// Output tiling of one fused launch.
struct Geometry {
    int tiles_x, tiles_y, chunks, chunk, out_x, out_y, halo_x, nblocks, threads;
    bool ok;
};

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

inline Geometry stream_geometry(int dim, int r, int k, VariantShape v, int64_t n0, int64_t n1,
                                int64_t n2, int chunk) {
    Geometry g{};
    g.threads = 64 * v.nw;
    g.halo_x = round_up(k * r, v.vx);
    g.out_x = 64 * v.vx - 2 * g.halo_x;
    g.out_y = (dim == 3) ? v.nw * v.rw - 2 * k * r : 1;
    if (g.out_x <= 0 || g.out_y <= 0) return g;
    g.tiles_x = (int)((n2 + g.out_x - 1) / g.out_x);
    g.tiles_y = (dim == 3) ? (int)((n1 + g.out_y - 1) / g.out_y) : 1;
    int64_t nxy = (dim == 3) ? (int64_t)g.tiles_x * g.tiles_y : (g.tiles_x + v.nw - 1) / v.nw;
    if (chunk <= 0) {
        // aim at ~2048 workgroups, keeping the per-chunk fill (K*(2R+1) extra
        // steps) below a quarter of the chunk
        int64_t want = (2048 + nxy - 1) / nxy;
        int64_t c = (n0 + want - 1) / want;
        int64_t cmin = 4 * (int64_t)k * (2 * r + 1);
        if (c < cmin) c = cmin;
        if (c > n0) c = n0;
        chunk = (int)c;
    }
    g.chunk = chunk;
    g.chunks = (int)((n0 + chunk - 1) / chunk);
    const int64_t nb = nxy * g.chunks;
    if (nb <= 0 || nb > 0x7fffffff) return g;
    g.nblocks = (int)nb;
    g.ok = true;
    return g;
}

// Chunk of the streamed axis that balances the launch over `resident`
// co-resident workgroups: a workgroup's time grows with its stream length
// (chunk + K(2R+1) steps of fill and drain) and the launch takes
// ceil(blocks / resident) rounds of workgroups, so pick the number of chunks
// that minimises rounds x stream length (fewer chunks on ties).  0 if the
// residency is unknown.
inline int balanced_chunk(int dim, int r, int k, VariantShape v, int64_t n0, int64_t n1, int64_t n2,
                          int resident) {
    if (resident <= 0 || dim < 2) return 0;
    const Geometry g = stream_geometry(dim, r, k, v, n0, n1, n2, (int)(n0 < 0x7fffffff ? n0 : 0x7fffffff));
    if (!g.ok) return 0;
    const int64_t nxy = g.nblocks;  // one chunk
    const int64_t fill = (int64_t)k * (2 * r + 1);
    const int64_t cmin = 2 * fill > 8 ? 2 * fill : 8;
    int64_t best_c = n0, best_cost = -1;
    const int64_t max_chunks = n0 / cmin > 1 ? n0 / cmin : 1;
    for (int64_t nc = 1; nc <= max_chunks && nc <= 4096; ++nc) {
        const int64_t c = (n0 + nc - 1) / nc;
        const int64_t chunks = (n0 + c - 1) / c;
        const int64_t rounds = (nxy * chunks + resident - 1) / resident;
        const int64_t cost = rounds * (c + fill);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best_c = c;
        }
    }
    return (int)best_c;
}

// y tiling of a tessellated 3D sweep: tiles of `tile_h` rows (the stage-A
// frame), the last starting at last_start; every tile must hold at least
// 2(K+1)R rows (its trapezoid and both slopes), so a short remainder is merged
// with the tile before it and the pair split in two.
struct TessTiling {
    int tile_h, tiles_y, last_start, ncut;
    bool ok;
};
inline TessTiling tess_tiling(int r, int k, int tile_h, int64_t n1, int bc) {
    TessTiling t{tile_h, 0, 0, 0, false};
    const int64_t need = 2 * (int64_t)(k + 1) * r;
    if (tile_h < need || n1 < need || n1 > 0x7fffffff) return t;
    int64_t tiles = (n1 + tile_h - 1) / tile_h;
    int64_t last = (tiles - 1) * tile_h;
    if (n1 - last < need) {
        if (tiles == 1) return t;
        // the last two tiles share their rows evenly
        const int64_t a = (tiles - 2) * tile_h;
        last = a + (n1 - a + 1) / 2;
        if (last - a < need || n1 - last < need) return t;
    }
    t.tiles_y = (int)tiles;
    t.last_start = (int)last;
    t.ncut = (int)tiles + (bc == 0 ? 1 : 0);  // the zero halo also cuts at n1
    t.ok = true;
    return t;
}

// slope buffer of a tessellated pass of k steps (compute-type elements)
inline int64_t tess_slope_bytes(int r, int k, int tile_h, int64_t n0, int64_t n1, int64_t n2, int bc,
                                int elem) {
    const TessTiling t = tess_tiling(r, k, tile_h, n1, bc);
    if (!t.ok || k < 2) return 0;
    return (int64_t)(k - 1) * t.tiles_y * 2 * n0 * 2 * r * n2 * elem;
}

// Rows of FP64 gradient partials a fused adjoint launch writes (one per wave).
inline int64_t adjoint_part_rows(int dim, int r, int k, VariantShape v, int64_t n0, int64_t n1, int64_t n2,
                                 int chunk) {
    const Geometry g = stream_geometry(dim, r, k, v, n0, n1, n2, chunk);
    return g.ok ? (int64_t)g.nblocks * v.nw : 0;
}

// Side buffer of one in-place pass (storage-type elements): per band block
// (one per workgroup and output plane; 2D: per wave) the band points of the
// output tile, then per whole-plane block (2*K*R per workgroup) a full tile.
struct InplaceSide {
    int64_t band, zplane, z0, total;
    bool ok;
};
inline InplaceSide inplace_side(int dim, int r, int k, VariantShape v, int64_t n0, int64_t n1, int64_t n2,
                                int chunk) {
    InplaceSide s{0, 0, 0, 0, false};
    const Geometry g = stream_geometry(dim, r, k, v, n0, n1, n2, chunk);
    if (!g.ok) return s;
    const int64_t subs = dim == 3 ? g.nblocks : (int64_t)g.nblocks * v.nw;
    const int64_t kr = (int64_t)k * r;
    s.band = dim == 3 ? 2 * kr * g.out_x + (int64_t)g.out_y * 2 * g.halo_x : 2 * (int64_t)g.halo_x;
    s.zplane = dim == 3 ? (int64_t)g.out_x * g.out_y : g.out_x;
    s.z0 = subs * g.chunk * s.band;
    s.total = s.z0 + subs * 2 * kr * s.zplane;
    s.ok = true;
    return s;
}

inline Geometry seg1d_geometry(int r, int k, VariantShape v, int64_t n) {
    Geometry g{};
    g.threads = 64 * v.nw;
    g.halo_x = round_up(k * r, v.vx);
    g.out_x = 64 * v.vx - 2 * g.halo_x;
    if (g.out_x <= 0) return g;
    const int64_t tiles = (n + g.out_x - 1) / g.out_x;
    if (tiles > 0x7fffffff) return g;
    g.tiles_x = (int)tiles;
    g.tiles_y = 1;
    g.chunks = 1;
    g.chunk = 1;
    g.out_y = 1;
    g.nblocks = (g.tiles_x + v.nw - 1) / v.nw;
    g.ok = g.nblocks > 0;
    return g;
}

// Registry lookups, defined in the instantiation units.  Return nullptr
// when no kernel is compiled for the combination.
SweepLauncher find_stream(int dtype, int dim, int r, bool box, int variant, int k);
SweepLauncher find_seg1d(int dtype, int r, int variant, int k);
bool variant_shape(int dim, int variant, VariantShape *out);
int num_variants(int dim);
int max_fused_k(int dim);

hipError_t launch_generic(int dtype, const void *src, void *dst, int64_t n0, int64_t n1,
                          int64_t n2, int npts, int bc, const int *d_off, const void *d_coef,
                          hipStream_t st);

}  // namespace stn
