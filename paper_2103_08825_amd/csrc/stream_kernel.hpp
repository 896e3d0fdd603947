// stream_kernel.hpp -- fused multi-step stencil sweep for 2D and 3D grids.
//
// One launch advances the grid by K time steps (the GPU counterpart of the
// time-loop unroll-and-jam of Section 3.3 / Algorithm 1: data is loaded once,
// advanced K steps on chip, and stored once, so bytes moved per point-step
// fall K-fold).
//
// Mapping (3D, axes z y x with x unit-stride; 2D is the same with no y):
//   * a workgroup owns an output tile out_x * out_y of the x-y plane and a
//     chunk of z; it holds the tile widened by a halo of K*R (overlapped
//     tiling: the halo is recomputed, shrinking by R per level);
//   * lane l of each 64-wide wave holds VX consecutive x columns; wave w of
//     the NW waves holds RW consecutive y rows;
//   * the workgroup streams the chunk plane by plane along z.  Level 0 is the
//     loaded plane; level j (1..K) keeps a ring of 2R+1 partial sums, one per
//     pending output plane.  When level j-1 delivers plane m, level j adds
//     plane m's in-plane weighted sums for every dz into output planes m-dz,
//     then plane m-R of level j is complete.  This is the pipeline of
//     Algorithm 1 turned sideways: the vector sets VS_1..VS_k in flight at
//     different time levels become the K rings, the booting and epilogue
//     computations become the fill and drain of the z stream;
//   * x neighbours come from the lane's own registers or from the adjacent
//     lane through whole-wave DPP shifts; y neighbours from the thread's own
//     rows, or, for the R rows at a wave's edge, from the adjacent wave
//     through a small double-buffered LDS halo written once per step.
//   * zero halo: every level forces points outside the grid to 0 (the
//     virtual halo is 0 at every step, also for the recomputed tile halo);
//     periodic: loads wrap per axis and nothing is masked.
#pragma once

#include "device_common.hpp"
#include "kernel_args.hpp"

namespace stn {

template <int DIM, int R, bool BOX, int DZ, int DY, int DX> constexpr bool is_member() {
    if constexpr (BOX) {
        return true;
    } else {
        return ((DZ != 0) + (DY != 0) + (DX != 0)) <= 1;
    }
}

template <int DIM, int R, int DZ, int DY, int DX> constexpr int dense_index() {
    constexpr int W = 2 * R + 1;
    if constexpr (DIM == 3) {
        return ((DZ + R) * W + (DY + R)) * W + (DX + R);
    } else {
        return (DZ + R) * W + (DX + R);
    }
}

// value at column (own column V) + DX of a row held as VX columns per lane
template <int DX, int V, int VX, typename C> __device__ __forceinline__ C xval(const C (&row)[VX]) {
    constexpr int t = V + DX;
    constexpr int s = floordiv(t, VX);
    constexpr int m = t - s * VX;
    return lane_shift<s>(row[m]);
}

// One workgroup's share of a fused launch: logical block `blk` of the grid
// described by `a`.  Called by stream_kernel (one block per workgroup) and by
// the persistent batched kernel (one block per work item).
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW>
__device__ __forceinline__ void stream_tile(const StreamArgs<typename ComputeOf<S>::type> &a, const int blk) {
    using C = typename ComputeOf<S>::type;
    constexpr int W = 2 * R + 1;
    constexpr int EXT = (DIM == 3) ? RW + 2 * R : 1;
    constexpr bool XCH = (DIM == 3) && (NW > 1);
    constexpr int YR = (DIM == 3) ? R : 0;
    static_assert(DIM == 2 || DIM == 3, "streaming kernel is for 2D and 3D grids");
    static_assert(DIM == 3 || RW == 1, "2D tiles hold one row per wave");

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wvu = __builtin_amdgcn_readfirstlane(wv);  // the wave's index, in a scalar register
    const S *__restrict__ src = static_cast<const S *>(a.src);
    S *__restrict__ dst = static_cast<S *>(a.dst);
    const bool periodic = (a.bc == 1);

    // ---- which tile ---------------------------------------------------------
    int tx, ty, zc;
    if constexpr (DIM == 3) {
        tx = blk % a.tiles_x;
        const int rest = blk / a.tiles_x;
        ty = rest % a.tiles_y;
        zc = rest / a.tiles_y;
    } else {
        const int groups = (a.tiles_x + NW - 1) / NW;
        tx = (blk % groups) * NW + wv;
        zc = blk / groups;
        ty = 0;
        if (tx >= a.tiles_x) return;  // 2D waves are independent: no barrier inside
    }
    const int64_t n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int64_t plane = n1 * n2;

    // ---- per-thread columns and rows (fixed along the stream) ----------------
    // The host guarantees n2 % VX == 0 and tile origins on multiples of VX, so
    // a lane's VX columns are either all inside the grid or all outside.  Each
    // row gets one 32-bit byte offset inside a plane; rows or columns outside
    // the grid (zero halo) or outside the output tile (stores) get an offset
    // past the end of the plane, which the buffer instructions turn into a
    // zero load or a dropped store.
    const int64_t x_out0 = (int64_t)tx * a.out_x;
    const int64_t x_base = x_out0 - a.halo_x;
    const int64_t x_lane = x_base + (int64_t)lane * VX;
    const bool x_inside = (x_lane >= 0) && (x_lane < n2);
    const bool x_in = periodic || x_inside;
    const int64_t x_eff = periodic ? wrap_index(x_lane, n2) : x_lane;
    const bool x_out = (x_lane >= x_out0) && (x_lane < x_out0 + a.out_x) && x_inside;
    const int64_t y_base = (DIM == 3) ? (int64_t)ty * a.out_y - K * R : 0;
    uint32_t ld_off[RW];  // byte offset of the lane's VX columns in each row (load)
    uint32_t st_off[RW];  // same for the store, or out of range
    bool y_in[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        int64_t ye = 0;
        bool y_ok = true, y_st = true;
        if constexpr (DIM == 3) {
            const int rel = wv * RW + i;  // row within the widened tile
            const int64_t y = y_base + rel;
            const bool inside = (y >= 0) && (y < n1);
            y_ok = periodic || inside;
            ye = periodic ? wrap_index(y, n1) : y;
            y_st = (rel >= K * R) && (rel < K * R + a.out_y) && inside;
        }
        y_in[i] = y_ok;
        const uint32_t off = (uint32_t)((ye * n2 + x_eff) * (int64_t)sizeof(S));
        ld_off[i] = (y_ok && x_in) ? off : kOutOfRange;
        st_off[i] = (y_st && x_out) ? off : kOutOfRange;
    }
    const uint32_t plane_bytes = (uint32_t)(plane * (int64_t)sizeof(S));

    // ---- z chunk (the streamed extent is below 2^31, checked on the host) -------
    const int nz = (int)n0;
    const int z_out0 = zc * a.chunk;
    const int z_out1 = (z_out0 + a.chunk < nz) ? z_out0 + a.chunk : nz;
    const int zs = z_out0 - K * R;  // plane loaded at step 0
    const int nload = (z_out1 - z_out0) + 2 * K * R;
    const int nsteps = (z_out1 - z_out0) + K * W;
    // Zero halo: a completed level plane must read 0 outside the grid.  If the
    // widened tile and every plane the chunk's outputs depend on lie inside the
    // grid, nothing needs masking (the common case); otherwise each completed
    // plane is masked with one select per point.
    const bool inside_xy = (x_base >= 0) && (x_base + 64 * VX <= n2) &&
                           (DIM == 2 || ((y_base >= 0) && (y_base + NW * RW <= n1)));
    const bool no_mask = periodic || (inside_xy && zs >= 0 && z_out1 + K * R <= nz);

    // ---- state ------------------------------------------------------------------
    C acc[K][W][RW][VX];  // level j+1's ring of pending output planes
    C pf[W][RW][VX];      // level-0 planes: plane p in slot p mod W
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int q = 0; q < W; ++q)
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int v = 0; v < VX; ++v) acc[j][q][i][v] = C(0);

    constexpr int kHaloLevels = XCH ? K : 1;
    constexpr int kHaloWaves = XCH ? NW : 1;
    constexpr int kHaloRows = XCH ? R : 1;
    constexpr int kHaloLanes = XCH ? 64 * VX : 1;
    __shared__ C halo[2][kHaloLevels][kHaloWaves][2][kHaloRows][kHaloLanes];

    // next plane to fetch: stream index, (wrapped) grid plane and its base
    int ld_s = 0;
    int ld_z = periodic ? (int)wrap_index(zs, nz) : zs;
    const S *ld_p = src + (int64_t)(ld_z > 0 ? ld_z : 0) * plane;

    auto load_next = [&](C (&out)[RW][VX]) {
        const bool z_ok = (ld_s < nload) && (periodic || (ld_z >= 0 && ld_z < nz));
        const rsrc_t r = make_rsrc(ld_p, z_ok ? plane_bytes : 0u);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const VecS<S, VX> t = vec_load<S, VX>(r, ld_off[i]);
#pragma unroll
            for (int v = 0; v < VX; ++v) out[i][v] = to_compute(t.v[v]);
        }
        ++ld_s;
        ++ld_z;
        if (ld_z > 0) ld_p += plane;
        if (periodic && ld_z == nz) {
            ld_z = 0;
            ld_p = src;
        }
    };

    auto store_plane = [&](int z, const C (&val)[RW][VX]) {
        const rsrc_t r = make_rsrc(dst + (int64_t)z * plane, plane_bytes);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            VecS<S, VX> t;
#pragma unroll
            for (int v = 0; v < VX; ++v) t.v[v] = from_compute<S>(val[i][v]);
            vec_store<S, VX>(t, r, st_off[i]);
        }
    };

    // one step of the stream; PH = s mod W selects ring slots at compile time
    auto step = [&](auto PH_, auto MASK_, int s) {
        constexpr int PH = decltype(PH_)::value;
        constexpr bool MASK = decltype(MASK_)::value;
        const int rd = (s + 1) & 1;  // LDS slot written by the previous step
        const int wr = s & 1;

        // levels K..1, each consuming the plane its predecessor delivered last step
        static_for<0, K>([&](auto JJ) {
            constexpr int j = K - decltype(JJ)::value;  // level 1..K
            constexpr int in_slot = posmod(PH - 1 - (j - 1) * (R + 1), W);
            // Skip work no kept point depends on (uniform branches): the incoming
            // plane feeds level-j planes [q, q+2R], q = the plane completed now; level
            // j is needed only on [z_out0 - (K-j)R, z_out1 - 1 + (K-j)R].  A wave whose
            // rows all lie within j*R of the widened tile's y edge holds only
            // recomputed halo at level j.  Measured: worth it for order-2 stencils;
            // for order 1 the branches cost more (they split the step into blocks the
            // scheduler cannot interleave) than the skipped work saves.
            constexpr bool kSkip = (R >= 2);
            const int q = zs + s - j * (R + 1);
            const bool needed = (q <= z_out1 - 1 + (K - j) * R) && (q + 2 * R >= z_out0 - (K - j) * R);
            const bool wave_on = (DIM == 2) || ((wvu + 1) * RW > j * R && wvu * RW < NW * RW - j * R);
            const bool work = !kSkip || (needed && wave_on);
            C ext[EXT][VX];
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    if constexpr (j == 1)
                        ext[YR + i][v] = pf[in_slot][i][v];  // level-0 plane s-1
                    else
                        ext[YR + i][v] = acc[j - 2][in_slot][i][v];
                }
            if constexpr (DIM == 3) {
#pragma unroll
                for (int e = 0; e < R; ++e)
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        // the first and last wave read their own rows instead of a
                        // missing neighbour: those rows lie outside the widened tile,
                        // whose edge is recomputed garbage that no kept point reads
                        C above = C(0), below = C(0);
                        if constexpr (XCH) {
                            const int wa = wv > 0 ? wv - 1 : 0;
                            const int wb = wv < NW - 1 ? wv + 1 : NW - 1;
                            above = halo[rd][j - 1][wa][1][e][lane * VX + v];
                            below = halo[rd][j - 1][wb][0][e][lane * VX + v];
                        }
                        ext[e][v] = above;
                        ext[R + RW + e][v] = below;
                    }
            }
            if constexpr (j == 1) {
                // slot of plane s-1 is free again: fetch plane s-1+W into it
                load_next(pf[in_slot]);
            }
            if constexpr (kSkip) {
                if (!work) return;
            }
            // FP64: lane-shifted copies of every row, shared by all their uses
            // (xs[e][v][dx+R] = row e at column v+dx); FP32 shifts inside each FMA
            constexpr bool kShareShifts = sizeof(C) == 8;
            C xs[kShareShifts ? EXT : 1][VX][W];
            if constexpr (kShareShifts) {
                static_for<0, EXT>([&](auto E_) {
                    constexpr int E = decltype(E_)::value;
                    static_for<0, VX>([&](auto V_) {
                        constexpr int V = decltype(V_)::value;
                        static_for<-R, R + 1>([&](auto DX_) {
                            constexpr int DX = decltype(DX_)::value;
                            xs[E][V][DX + R] = xval<DX, V, VX>(ext[E]);
                        });
                    });
                });
            }
            // scatter plane m into output planes m-dz of level j.  Every point's
            // terms are added in the canonical offset order; the loop runs over
            // offsets outside and rows inside, so the rows' lane-shifted terms of
            // one offset issue together.
            static_for<-R, R + 1>([&](auto DZ_) {
                constexpr int DZ = decltype(DZ_)::value;
                constexpr int slot = posmod(PH - 1 - (j - 1) * (R + 1) - DZ, W);
                C t[VX][RW];
#pragma unroll
                for (int i = 0; i < RW; ++i)
#pragma unroll
                    for (int v = 0; v < VX; ++v) t[v][i] = (DZ == -R) ? C(0) : acc[j - 1][slot][i][v];
                static_for<-YR, YR + 1>([&](auto DY_) {
                    constexpr int DY = decltype(DY_)::value;
                    static_for<-R, R + 1>([&](auto DX_) {
                        constexpr int DX = decltype(DX_)::value;
                        if constexpr (is_member<DIM, R, BOX, DZ, DY, DX>()) {
                            const C c = a.coef[dense_index<DIM, R, DZ, DY, DX>()];
                            static_for<0, VX>([&](auto V_) {
                                constexpr int V = decltype(V_)::value;
                                constexpr int sh = floordiv(V + DX, VX);  // lanes away
                                constexpr int m = V + DX - sh * VX;        // column in that lane
                                if constexpr (kShareShifts) {
#pragma unroll
                                    for (int i = 0; i < RW; ++i) t[V][i] = fma_c(c, xs[YR + i + DY][V][DX + R], t[V][i]);
                                } else if constexpr (sh == 0) {
#pragma unroll
                                    for (int i = 0; i < RW; ++i) t[V][i] = fma_c(c, ext[YR + i + DY][m], t[V][i]);
                                } else {
                                    C x[RW];
#pragma unroll
                                    for (int i = 0; i < RW; ++i) x[i] = ext[YR + i + DY][m];
                                    fma_shift_rows<sh, RW>(c, x, t[V]);
                                }
                            });
                        }
                    });
                });
#pragma unroll
                for (int i = 0; i < RW; ++i)
#pragma unroll
                    for (int v = 0; v < VX; ++v) acc[j - 1][slot][i][v] = t[v][i];
            });
            // plane m-R of level j is complete: apply the zero halo
            if constexpr (j < K && MASK) {
                constexpr int cslot = posmod(PH - j * (R + 1), W);
                const int z = zs + s - j * (R + 1);
                const bool z_ok = (z >= 0) && (z < nz);
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const bool keep = z_ok && y_in[i] && x_in;
#pragma unroll
                    for (int v = 0; v < VX; ++v) acc[j - 1][cslot][i][v] = keep ? acc[j - 1][cslot][i][v] : C(0);
                }
            }
        });

        // publish the edge rows of every plane delivered this step (level 0: plane s)
        if constexpr (XCH) {
            static_for<0, K>([&](auto L_) {
                constexpr int lvl = decltype(L_)::value;  // 0..K-1
                constexpr int cslot = posmod(PH - lvl * (R + 1), W);
#pragma unroll
                for (int e = 0; e < R; ++e)
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        C top, bot;
                        if constexpr (lvl == 0) {
                            top = pf[PH][e][v];
                            bot = pf[PH][RW - R + e][v];
                        } else {
                            top = acc[lvl - 1][cslot][e][v];
                            bot = acc[lvl - 1][cslot][RW - R + e][v];
                        }
                        halo[wr][lvl][wv][0][e][lane * VX + v] = top;
                        halo[wr][lvl][wv][1][e][lane * VX + v] = bot;
                    }
            });
        }

        // level K delivered an output plane
        {
            constexpr int oslot = posmod(PH - K * (R + 1), W);
            const int z = zs + s - K * (R + 1);
            if (z >= z_out0 && z < z_out1) store_plane(z, acc[K - 1][oslot]);
        }
        if constexpr (XCH) __syncthreads();
    };

    // prologue: planes 0..W-2 in flight; slot W-1 stands for plane -1 (zero)
#pragma unroll
    for (int q = 0; q < W - 1; ++q) load_next(pf[q]);
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int v = 0; v < VX; ++v) pf[W - 1][i][v] = C(0);
    // With kWholeBlocks the stream runs in whole blocks of W steps (up to W-1
    // steps past its end, which load and store nothing).  A partial last block
    // makes the ring slots conditional at the loop back-edge; the register copies
    // that merge them wait for the loads in flight, which shortens the prefetch,
    // but they also bound the registers the loads hold.  Measured on 512^3: whole
    // blocks win for the 27-point box and the order-2 star (5-9%); for the FP32
    // 7-point star they push the deeper fused kernels into spills, and they cost
    // FP64 and 16-bit storage a few per cent.
    constexpr bool kWholeBlocks = (BOX || R >= 2) && sizeof(C) == 4;
    auto run = [&](auto MASK_) {
        for (int s0 = 0; s0 < nsteps; s0 += W) {
            static_for<0, W>([&](auto PH_) {
                const int s = s0 + decltype(PH_)::value;
                if constexpr (kWholeBlocks) {
                    step(PH_, MASK_, s);
                } else {
                    if (s < nsteps) step(PH_, MASK_, s);
                }
            });
        }
    };
    if (no_mask)
        run(std::integral_constant<bool, false>{});
    else
        run(std::integral_constant<bool, true>{});
}

template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW>
__global__ void __launch_bounds__(64 * NW)
    stream_kernel(const StreamArgs<typename ComputeOf<S>::type> a) {
    stream_tile<S, DIM, R, BOX, K, VX, NW, RW>(a, xcd_remap(blockIdx.x, a.nblocks));
}

}  // namespace stn
