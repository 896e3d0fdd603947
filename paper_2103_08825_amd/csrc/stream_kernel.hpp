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
//   * zero halo: star stencils give weight 0 to every term whose neighbour
//     lies outside the grid; box stencils force every point outside the grid
//     to 0 at every level (the virtual halo is 0 at every step, also for the
//     recomputed tile halo); periodic: loads wrap per axis, nothing is masked.
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

// Launch modes of the streaming kernel.
//   kOverlapped: the fused sweep above (tiles widened by a recomputed halo).
//   kTessA, kTessB: the two stages of a tessellated fused sweep (Section 3.4),
//     tessellating the y axis (rows are held per wave, so rows outside a
//     level's valid region can be skipped whole) while x stays overlapped
//     (lanes) and z stays streamed.  The y axis is cut into tiles; stage A
//     advances every tile by K levels on a shrinking trapezoid (level j valid on
//     the tile's rows [jR, h - jR)), stores the finished rows [KR, h - KR) and,
//     for every level L < K, the 2R rows on each side that the next stage
//     needs (the slopes: rows [LR, (L+2)R) and [h-(L+2)R, h-LR)).  Stage B
//     advances the inverted trapezoid around every cut c (level j valid on
//     [c - jR, c + jR)), taking the rows beyond its own valid region from the
//     stored slopes, and stores the rows [c - KR, c + KR).  After stage A each
//     row of a tile has advanced min(d, K) levels, d = its distance in rows/R to
//     the nearer cut, which is the triangle state pattern of Section 3.4;
//     stage B adds the complement.  Intermediate levels are kept (and stored
//     as slopes) in compute precision, so the result equals the overlapped
//     sweep's bit for bit.
//   kInPlace: the fused sweep with src == dst.  Every point another workgroup
//     reads (its widened tile reaches halo_x columns, K*R rows and K*R planes
//     into ours) is a band point of our output region: band points go to a
//     side buffer and a second kernel copies them into the field once every
//     workgroup has read its inputs; the other points are written in place
//     (no other workgroup reads them, and this one read them before).
//   kAdjoint: K steps of the mirrored stencil (the dense table reversed on
//     the host) from lambda_{t+1} to lambda_{t+1-K}, with the coefficient
//     gradient folded in: level j (time s = t+1-j) reads lambda_{s+1} as
//     level j-1 and the forward state u_s (ustate[j-1]), and adds
//     u_s[y] * lambda_{s+1}[y + d] for every term d of the mirrored stencil
//     and every point y the workgroup owns (its output tile and chunk).  The
//     term d pairs with the canonical offset o = -d, so partial row entry
//     npts-1-t (t: the term's rank in the kernel's lexicographic order) is
//     dL/dc for that offset.  FP64 plans form and sum the products in FP64;
//     FP32 plans sum a step's products in FP32 (rounding each product once,
//     a few products per sum) and fold them into FP64 sums every step.
//   kLevels: the fused sweep that also stores every intermediate level
//     (level j < K to ustate[j-1], level K to dst): the states a segment of
//     the adjoint recomputes, K of them per launch.
enum : int { kOverlapped = 0, kTessA = 1, kTessB = 2, kInPlace = 3, kAdjoint = 4, kLevels = 5 };

// rank of term (DZ, DY, DX) among the stencil's members in lexicographic order
template <int DIM, int R, bool BOX, int DZ, int DY, int DX> constexpr int term_rank() {
    constexpr int YR = DIM == 3 ? R : 0;
    int n = 0;
    for (int dz = -R; dz <= R; ++dz)
        for (int dy = -YR; dy <= YR; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
                if (dz == DZ && dy == DY && dx == DX) return n;
                const bool member = BOX || ((dz != 0) + (dy != 0) + (dx != 0)) <= 1;
                n += member;
            }
    return n;
}
template <int DIM, int R, bool BOX> constexpr int num_terms() {
    constexpr int YR = DIM == 3 ? R : 0;
    int n = 0;
    for (int dz = -R; dz <= R; ++dz)
        for (int dy = -YR; dy <= YR; ++dy)
            for (int dx = -R; dx <= R; ++dx) n += BOX || ((dz != 0) + (dy != 0) + (dx != 0)) <= 1;
    return n;
}

// One workgroup's share of a fused launch: logical block `blk` of the grid
// described by `a`.  Called by stream_kernel (one block per workgroup) and by
// the persistent batched kernel (one block per work item).
template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW, int MODE = kOverlapped>
__device__ __forceinline__ void stream_tile(const StreamArgs<typename ComputeOf<S>::type> &a, const int blk) {
    using C = typename ComputeOf<S>::type;
    constexpr int W = 2 * R + 1;
    constexpr int EXT = (DIM == 3) ? RW + 2 * R : 1;
    constexpr bool XCH = (DIM == 3) && (NW > 1);
    constexpr int YR = (DIM == 3) ? R : 0;
    static_assert(DIM == 2 || DIM == 3, "streaming kernel is for 2D and 3D grids");
    static_assert(DIM == 3 || RW == 1, "2D tiles hold one row per wave");
    static_assert(!(MODE == kTessA || MODE == kTessB) || DIM == 3, "the tessellated stages are for 3D grids");
    // the fused adjoint runs the stream in blocks of 2W steps: its forward-state
    // ring has 2W slots, filled W steps ahead of use
    constexpr int UNROLL = MODE == kAdjoint ? 2 * W : W;
    constexpr int WU = 2 * W;
    constexpr int NT = num_terms<DIM, R, BOX>();

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wvu = __builtin_amdgcn_readfirstlane(wv);  // the wave's index, in a scalar register
    const S *__restrict__ src = static_cast<const S *>(a.src);
    S *__restrict__ dst = static_cast<S *>(a.dst);
    const bool periodic = (a.bc == 1);

    // ---- which tile ---------------------------------------------------------
    int tx, ty, zc;
    if constexpr (DIM == 3) {
        const int ny = MODE == kTessB ? a.ncut : a.tiles_y;  // stage B: ty is the cut
        tx = blk % a.tiles_x;
        const int rest = blk / a.tiles_x;
        ty = rest % ny;
        zc = rest / ny;
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
    // tessellated y tiles start at multiples of tile_h except the last, which
    // starts at last_start; cut c lies at the start of tile c (also at n1 for
    // the zero halo)
    auto tile_start = [&](int t) -> int { return t >= a.tiles_y - 1 ? a.last_start : t * a.tile_h; };
    int tess_h = 0;  // stage A: rows of this tile
    int64_t y_base = 0;
    if constexpr (DIM == 3) {
        if constexpr (MODE == kTessA) {
            y_base = tile_start(ty);
            tess_h = (int)((ty + 1 < a.tiles_y ? (int64_t)tile_start(ty + 1) : n1) - y_base);
        } else if constexpr (MODE == kTessB) {
            y_base = (ty < a.tiles_y ? (int64_t)tile_start(ty) : n1) - (K + 1) * R;
        } else {
            y_base = (int64_t)ty * a.out_y - K * R;
        }
    }
    // rows of the frame stored at level K
    const int st_lo = MODE == kTessA ? K * R : (MODE == kTessB ? R : K * R);
    const int st_hi = MODE == kTessA ? tess_h - K * R : (MODE == kTessB ? R + 2 * K * R : K * R + a.out_y);
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
            // stage B's frame around the periodic cut at 0 stores wrapped rows;
            // elsewhere a frame row beyond the grid is a periodic image of a row
            // another tile stores, and is not stored
            y_st = (rel >= st_lo) && (rel < st_hi) && (inside || (MODE == kTessB && periodic));
        }
        y_in[i] = y_ok;
        const uint32_t off = (uint32_t)((ye * n2 + x_eff) * (int64_t)sizeof(S));
        ld_off[i] = (y_ok && x_in) ? off : kOutOfRange;
        st_off[i] = (y_st && x_out) ? off : kOutOfRange;
    }
    const uint32_t plane_bytes = (uint32_t)(plane * (int64_t)sizeof(S));

    // In place: band points of the output region (within halo_x columns or K*R
    // rows of its edge; planes within K*R of the chunk's ends are handled whole)
    // are stored to the side buffer instead of the field.  sd_off: offset in the
    // plane's band block, zd_off: offset in a whole-plane block.
    uint32_t sd_off[MODE == kInPlace ? RW : 1], zd_off[MODE == kInPlace ? RW : 1];
    if constexpr (MODE == kInPlace) {
        const int hx = a.halo_x;
        const int ow = (int)(n2 - x_out0 < a.out_x ? n2 - x_out0 : a.out_x);
        const int xr = (int)(x_lane - x_out0);
        const bool xband = xr < hx || xr >= ow - hx;
        const int oh = DIM == 3 ? (int)(n1 - (int64_t)ty * a.out_y < a.out_y ? n1 - (int64_t)ty * a.out_y : a.out_y) : 1;
        constexpr int KRY = DIM == 3 ? K * R : 0;  // band rows
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int yr = DIM == 3 ? wv * RW + i - K * R : 0;
            const bool top = yr < KRY, bot = !top && yr >= oh - KRY;
            int idx;
            if (top)
                idx = yr * ow + xr;
            else if (bot)
                idx = KRY * ow + (yr - (oh - KRY)) * ow + xr;
            else
                idx = 2 * KRY * ow + (yr - KRY) * 2 * hx + (xr < hx ? xr : hx + xr - (ow - hx));
            const bool out = st_off[i] != kOutOfRange;
            const bool band = top || bot || xband;
            sd_off[i] = (out && band) ? (uint32_t)idx * (uint32_t)sizeof(S) : kOutOfRange;
            zd_off[i] = out ? (uint32_t)(yr * a.out_x + xr) * (uint32_t)sizeof(S) : kOutOfRange;
            if (band) st_off[i] = kOutOfRange;
        }
    }

    // 3D star stencils take the zero halo through their weights: a term whose
    // neighbour lies outside the grid gets weight 0, so points outside the grid
    // may hold any finite value (they start at 0 and only ever receive weighted
    // sums of finite values) and no level needs masking.  The x test is per lane
    // and lane shift (a lane's VX columns are all inside or all outside), the y
    // test per row (uniform per wave), the z test per source plane (uniform per
    // step).  Box stencils mix axes in one term and keep the per-level masks;
    // so do 2D grids, whose waves hold one row: there the per-level scalar work
    // of the z test outweighs the row's few FMAs, while interior tiles of the
    // masked scheme need no mask at all.
    constexpr bool kWeightHalo = !BOX && DIM == 3;
    constexpr int SHX = (R + VX - 1) / VX;  // lane shifts an x neighbour can need
    const int pmask = -a.bc;                  // -1 periodic, 0 zero halo
    int xnb[2 * SHX + 1];                     // per lane: the neighbour lane is inside
#pragma unroll
    for (int sh = -SHX; sh <= SHX; ++sh) xnb[sh + SHX] = pmask | mask_in((int)x_lane + sh * VX, (int)n2);
    int ynb[RW][2 * YR + 1];                  // per row (wave-uniform): the neighbour row is inside
    const int y_wave = (int)y_base + wvu * RW;
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int dy = -YR; dy <= YR; ++dy) ynb[i][dy + YR] = pmask | mask_in(y_wave + i + dy, (int)n1);

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

    // fused adjoint: forward-state ring per level (output plane q in slot
    // (q - zs) mod 2W; 0 where this workgroup does not own the point) and the
    // thread's FP64 gradient sums per term
    C ur[MODE == kAdjoint ? K : 1][MODE == kAdjoint ? WU : 1][RW][VX];
    double gsum[MODE == kAdjoint ? NT : 1];
    // FP32 plans: a step's products (at most K*RW*VX per term) are summed in
    // FP32 and folded into the FP64 sums once per step
    C gstep[MODE == kAdjoint ? NT : 1];
    if constexpr (MODE == kAdjoint) {
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < WU; ++q)
#pragma unroll
                for (int i = 0; i < RW; ++i)
#pragma unroll
                    for (int v = 0; v < VX; ++v) ur[j][q][i][v] = C(0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            gsum[t] = 0.0;
            gstep[t] = C(0);
        }
    }

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
        const int z_ok = mask_lt(ld_s, nload) & (pmask | mask_in(ld_z, nz));
        const rsrc_t r = make_rsrc(ld_p, plane_bytes & (uint32_t)z_ok);
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
        VecS<S, VX> t[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i)
#pragma unroll
            for (int v = 0; v < VX; ++v) t[i].v[v] = from_compute<S>(val[i][v]);
        if constexpr (MODE == kInPlace) {
            S *const side = static_cast<S *>(a.slope);
            const int64_t sblk = DIM == 3 ? blk : (int64_t)blk * NW + wv;  // 2D: one x tile per wave
            const int zl = z - z_out0;
            if (zl < K * R || z >= z_out1 - K * R) {
                // a plane the neighbouring chunks read: the whole output tile to the side
                const int zb = zl < K * R ? zl : K * R + z - (z_out1 - K * R);
                const rsrc_t r = make_rsrc(side + a.side_z0 + (sblk * 2 * K * R + zb) * a.side_zplane,
                                           (uint32_t)(a.side_zplane * (int64_t)sizeof(S)));
#pragma unroll
                for (int i = 0; i < RW; ++i) vec_store<S, VX>(t[i], r, zd_off[i]);
                return;
            }
            const rsrc_t rb = make_rsrc(side + (sblk * a.chunk + zl) * a.side_band,
                                        (uint32_t)(a.side_band * (int64_t)sizeof(S)));
#pragma unroll
            for (int i = 0; i < RW; ++i) vec_store<S, VX>(t[i], rb, sd_off[i]);
        }
        const rsrc_t r = make_rsrc(dst + (int64_t)z * plane, plane_bytes);
#pragma unroll
        for (int i = 0; i < RW; ++i) vec_store<S, VX>(t[i], r, st_off[i]);
    };

    // ---- slopes of the tessellated stages -------------------------------------
    // Slope buffer (compute type): for level L in 1..K-1, tile t, plane z, side
    // (0: the tile's first rows, 1: its last rows), slope row 0..2R-1, column x:
    // element (((L-1) * tiles_y + t) * n0 + z) * 4R * n2 + (side * 2R + row) * n2 + x.
    // Per level and row of this thread, the byte offset of its slope row within
    // the (L, tile, z) block (the lane's column included), or out of range when
    // the row holds no slope row at that level.  Stage B reads the slopes of two
    // tiles: the one above the cut (its last rows) and the one below (its first).
    constexpr int NL = (MODE != kOverlapped && K > 1) ? K - 1 : 1;
    constexpr uint32_t kSlopeElem = sizeof(C);
    const uint32_t row_bytes = (uint32_t)(n2 * kSlopeElem);
    const uint32_t sx_st = x_out ? (uint32_t)(x_eff * kSlopeElem) : kOutOfRange;
    const uint32_t sx_ld = x_in ? (uint32_t)(x_eff * kSlopeElem) : kOutOfRange;
    uint32_t so_a[NL][RW];  // stage A: own tile; stage B: the tile above the cut
    uint32_t so_b[NL][RW];  // stage B: the tile below the cut
    int t_above = -1, t_below = -1;
    if constexpr (MODE == kTessB) {
        t_above = ty > 0 ? ty - 1 : (periodic ? a.tiles_y - 1 : -1);
        t_below = ty < a.tiles_y ? ty : -1;
    }
#pragma unroll
    for (int L = 1; L <= NL; ++L)
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int rel = wv * RW + i;
            uint32_t oa = kOutOfRange, ob = kOutOfRange;
            if constexpr (MODE == kTessA) {
                if (rel >= L * R && rel < (L + 2) * R)
                    oa = sx_st + (uint32_t)(rel - L * R) * row_bytes;  // side 0
                else if (rel >= tess_h - (L + 2) * R && rel < tess_h - L * R)
                    oa = sx_st + (uint32_t)(2 * R + rel - (tess_h - (L + 2) * R)) * row_bytes;  // side 1
            } else if constexpr (MODE == kTessB) {
                const int d = rel - (K + 1) * R;  // row relative to the cut
                const int64_t y = y_base + rel;
                const bool inside = periodic || (y >= 0 && y < n1);
                if (inside && t_above >= 0 && d >= -(L + 2) * R && d < -L * R)
                    oa = sx_ld + (uint32_t)(2 * R + d + (L + 2) * R) * row_bytes;  // above: its side 1
                if (inside && t_below >= 0 && d >= L * R && d < (L + 2) * R)
                    ob = sx_ld + (uint32_t)(d - L * R) * row_bytes;  // below: its side 0
            }
            so_a[L - 1][i] = oa;
            so_b[L - 1][i] = ob;
        }
    C *const slope = static_cast<C *>(a.slope);
    const int64_t slope_blk = 4 * R * n2;  // elements of one (level, tile, plane) block
    // rsrc of the (L, tile t, plane z) block; empty for a missing tile or a
    // plane outside the grid (zero halo), wrapped for the periodic rule
    auto slope_rsrc = [&](int L, int t, int z) -> rsrc_t {
        const int zz = periodic ? (int)wrap_index(z, nz) : z;
        const int ok = mask_in(t, a.tiles_y) & mask_in(zz, nz);
        const int64_t blk = ok ? (((int64_t)(L - 1) * a.tiles_y + t) * n0 + zz) * slope_blk : 0;
        return make_rsrc(slope + blk, (uint32_t)(slope_blk * kSlopeElem) & (uint32_t)ok);
    };
    // stage A: level L has completed plane z (slot cslot); store its slope rows
    auto tess_store = [&](auto L_, auto PH_, int s) {
        constexpr int L = decltype(L_)::value;
        constexpr int PH = decltype(PH_)::value;
        constexpr int cslot = posmod(PH - L * (R + 1), W);
        const int z = zs + s - L * (R + 1);
        if (z < z_out0 || z >= z_out1) return;  // each chunk stores its own planes
        // only the waves at the tile's edges hold slope rows
        const bool has_top = (wvu + 1) * RW > L * R && wvu * RW < (L + 2) * R;
        const bool has_bot = (wvu + 1) * RW > tess_h - (L + 2) * R && wvu * RW < tess_h - L * R;
        if (!has_top && !has_bot) return;
        const rsrc_t r = slope_rsrc(L, ty, z);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            VecS<C, VX> t;
#pragma unroll
            for (int v = 0; v < VX; ++v) t.v[v] = acc[L - 1][cslot][i][v];
            vec_store<C, VX>(t, r, so_a[L - 1][i]);
        }
    };
    // stage B: the slope rows of the plane level L completes at step s sit in
    // ring slot s mod W, loaded W steps ahead (a row takes the above tile's
    // value or the below tile's; the other load reads 0)
    C sl[MODE == kTessB ? NL : 1][W][RW][VX];
    auto tess_fetch = [&](auto L_, auto Q_, int s_use) {
        constexpr int L = decltype(L_)::value;
        constexpr int Q = decltype(Q_)::value;
        const int z = zs + s_use - L * (R + 1);
        const rsrc_t ra = slope_rsrc(L, t_above, z);
        const rsrc_t rb = slope_rsrc(L, t_below, z);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const VecS<C, VX> ta = vec_load<C, VX>(ra, so_a[L - 1][i]);
            const VecS<C, VX> tb = vec_load<C, VX>(rb, so_b[L - 1][i]);
#pragma unroll
            for (int v = 0; v < VX; ++v) sl[L - 1][Q][i][v] = bits_or(ta.v[v], tb.v[v]);
        }
    };
    auto tess_inject = [&](auto L_, auto PH_, int s) {
        constexpr int L = decltype(L_)::value;
        constexpr int PH = decltype(PH_)::value;
        constexpr int cslot = posmod(PH - L * (R + 1), W);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const bool take = (so_a[L - 1][i] != kOutOfRange) || (so_b[L - 1][i] != kOutOfRange);
#pragma unroll
            for (int v = 0; v < VX; ++v) acc[L - 1][cslot][i][v] = take ? sl[L - 1][PH][i][v] : acc[L - 1][cslot][i][v];
        }
        tess_fetch(L_, PH_, s + W);  // the slot is free again: fetch W steps ahead
    };

    // fused adjoint: level j's forward state at plane q into ring slot Q (owned
    // points only: the store offsets mark them; planes outside the chunk read 0)
    auto ustate_fetch = [&](auto J_, auto Q_, int q) {
        constexpr int J = decltype(J_)::value;
        constexpr int Q = decltype(Q_)::value;
        const S *u = static_cast<const S *>(a.ustate[J - 1]);
        const int own = mask_in(q - z_out0, z_out1 - z_out0);
        const rsrc_t r = make_rsrc(u + (int64_t)(own ? q : 0) * plane, plane_bytes & (uint32_t)own);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const VecS<S, VX> t = vec_load<S, VX>(r, st_off[i]);
#pragma unroll
            for (int v = 0; v < VX; ++v) ur[J - 1][Q][i][v] = to_compute(t.v[v]);
        }
    };

    // one step of the stream; PH = s mod UNROLL selects ring slots at compile time
    auto step = [&](auto PH_, auto MASK_, int s) {
        constexpr int PH = decltype(PH_)::value;
        // bit 0: mask every completed level (box stencils, zero halo); bit 1:
        // the fused adjoint's gradient skips neighbours outside the grid (star
        // stencils, zero halo)
        constexpr bool MASK = (decltype(MASK_)::value & 1) != 0;
        constexpr bool GMASK = (decltype(MASK_)::value & 2) != 0;
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
            // (The tessellated stages always skip: stage B's valid region is a
            // few rows wide at the low levels.)
            constexpr bool kSkip = (R >= 2) || MODE != kOverlapped;
            const int q = zs + s - j * (R + 1);
            const bool needed = (q <= z_out1 - 1 + (K - j) * R) && (q + 2 * R >= z_out0 - (K - j) * R);
            // rows of the frame valid at level j
            const int vlo = MODE == kTessB ? (K + 1 - j) * R : j * R;
            const int vhi = MODE == kTessB ? (K + 1 + j) * R : (MODE == kTessA ? tess_h - j * R : NW * RW - j * R);
            const bool wave_on = (DIM == 2) || ((wvu + 1) * RW > vlo && wvu * RW < vhi);
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
                if (!work) {
                    // stage B still takes this level's slope rows
                    if constexpr (MODE == kTessB && j < K) tess_inject(std::integral_constant<int, j>{}, PH_, s);
                    return;
                }
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
            const int m_src = zs + s - 1 - (j - 1) * (R + 1);  // the plane being scattered
            const int src_in = pmask | mask_in(m_src, nz);
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
                            const C c0 = a.coef[dense_index<DIM, R, DZ, DY, DX>()];
                            // weight of the term (zero-halo weights for star stencils)
                            const C c = (kWeightHalo && DZ != 0) ? weight_if(c0, src_in) : c0;
                            static_for<0, VX>([&](auto V_) {
                                constexpr int V = decltype(V_)::value;
                                constexpr int sh = floordiv(V + DX, VX);  // lanes away
                                constexpr int m = V + DX - sh * VX;        // column in that lane
                                const C cx = (kWeightHalo && sh != 0) ? weight_if(c, xnb[sh + SHX]) : c;
                                if constexpr (kShareShifts) {
#pragma unroll
                                    for (int i = 0; i < RW; ++i) {
                                        const C ci = (kWeightHalo && DY != 0) ? weight_if(cx, ynb[i][DY + YR]) : cx;
                                        t[V][i] = fma_c(ci, xs[YR + i + DY][V][DX + R], t[V][i]);
                                    }
                                } else if constexpr (sh == 0) {
#pragma unroll
                                    for (int i = 0; i < RW; ++i) {
                                        const C ci = (kWeightHalo && DY != 0) ? weight_if(cx, ynb[i][DY + YR]) : cx;
                                        t[V][i] = fma_c(ci, ext[YR + i + DY][m], t[V][i]);
                                    }
                                } else {
                                    C x[RW];
#pragma unroll
                                    for (int i = 0; i < RW; ++i) x[i] = ext[YR + i + DY][m];
                                    fma_shift_rows<sh, RW>(cx, x, t[V]);
                                }
                                if constexpr (MODE == kAdjoint) {
                                    // dL/dc: u_s at the output point times lambda_{s+1} at its
                                    // neighbour, where the neighbour lies inside the grid
                                    constexpr int TR = term_rank<DIM, R, BOX, DZ, DY, DX>();
                                    constexpr int us = posmod(PH - 1 - (j - 1) * (R + 1) - DZ, WU);
                                    int mk = -1;
                                    if constexpr (GMASK && DZ != 0) mk &= src_in;
                                    if constexpr (GMASK && sh != 0) mk &= xnb[sh + SHX];
                                    C uo[RW];
#pragma unroll
                                    for (int i = 0; i < RW; ++i) {
                                        int mi = mk;
                                        if constexpr (GMASK && DY != 0) mi &= ynb[i][DY + YR];
                                        uo[i] = (GMASK && (DZ != 0 || DY != 0 || sh != 0)) ? weight_if(ur[j - 1][us][i][V], mi)
                                                                                          : ur[j - 1][us][i][V];
                                    }
                                    if constexpr (sizeof(C) == 4 && !kShareShifts && (sh == 1 || sh == -1)) {
                                        // the neighbour in the adjacent lane as a DPP operand
                                        C x[RW];
#pragma unroll
                                        for (int i = 0; i < RW; ++i) x[i] = ext[YR + i + DY][m];
                                        dpp_fmac_chain<sh, RW>(uo, x, gstep[TR]);
                                    } else {
#pragma unroll
                                        for (int i = 0; i < RW; ++i) {
                                            C nb;
                                            if constexpr (kShareShifts)
                                                nb = xs[YR + i + DY][V][DX + R];
                                            else
                                                nb = lane_shift<sh>(ext[YR + i + DY][m]);
                                            if constexpr (sizeof(C) == 8)
                                                gsum[TR] = __builtin_fma(uo[i], nb, gsum[TR]);
                                            else
                                                gstep[TR] = fma_c(uo[i], nb, gstep[TR]);
                                        }
                                    }
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
            if constexpr (MODE == kTessA && j < K) tess_store(std::integral_constant<int, j>{}, PH_, s);
            if constexpr (MODE == kLevels && j < K) {
                // level j has completed plane z: store it like an output plane
                constexpr int cslot = posmod(PH - j * (R + 1), W);
                const int z = zs + s - j * (R + 1);
                if (z >= z_out0 && z < z_out1) {
                    S *lv = static_cast<S *>(const_cast<void *>(a.ustate[j - 1]));
                    const rsrc_t r = make_rsrc(lv + (int64_t)z * plane, plane_bytes);
#pragma unroll
                    for (int i = 0; i < RW; ++i) {
                        VecS<S, VX> t;
#pragma unroll
                        for (int v = 0; v < VX; ++v) t.v[v] = from_compute<S>(acc[j - 1][cslot][i][v]);
                        vec_store<S, VX>(t, r, st_off[i]);
                    }
                }
            }
            if constexpr (MODE == kTessB && j < K) tess_inject(std::integral_constant<int, j>{}, PH_, s);
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
                            top = pf[PH % W][e][v];
                            bot = pf[PH % W][RW - R + e][v];
                        } else {
                            top = acc[lvl - 1][cslot][e][v];
                            bot = acc[lvl - 1][cslot][RW - R + e][v];
                        }
                        halo[wr][lvl][wv][0][e][lane * VX + v] = top;
                        halo[wr][lvl][wv][1][e][lane * VX + v] = bot;
                    }
            });
        }

        // fused adjoint: fold the step's FP32 gradient sums; fetch each level's
        // forward state for the plane that becomes pending W steps from now (its
        // slot was freed by the previous step)
        if constexpr (MODE == kAdjoint && sizeof(C) == 4) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                gsum[t] += (double)gstep[t];
                gstep[t] = C(0);
            }
        }
        if constexpr (MODE == kAdjoint) {
            static_for<1, K + 1>([&](auto J_) {
                constexpr int J = decltype(J_)::value;
                constexpr int Q = posmod(PH + W - 1 - (J - 1) * (R + 1) + R, WU);
                ustate_fetch(J_, std::integral_constant<int, Q>{}, zs + s + W - 1 - (J - 1) * (R + 1) + R);
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
    if constexpr (MODE == kTessB) {
        static_for<1, K>([&](auto L_) {
            static_for<0, W>([&](auto Q_) { tess_fetch(L_, Q_, decltype(Q_)::value); });
        });
    }
    if constexpr (MODE == kAdjoint) {
        // the planes that become pending in the first W steps
        static_for<1, K + 1>([&](auto J_) {
            constexpr int J = decltype(J_)::value;
            static_for<0, W>([&](auto T_) {
                constexpr int T0 = decltype(T_)::value;
                constexpr int Q = posmod(T0 - 1 - (J - 1) * (R + 1) + R, WU);
                ustate_fetch(J_, std::integral_constant<int, Q>{}, zs + T0 - 1 - (J - 1) * (R + 1) + R);
            });
        });
    }
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
    constexpr bool kWholeBlocks = (BOX || R >= 2 || MODE == kLevels) && sizeof(C) == 4;
    auto run = [&](auto MASK_) {
        for (int s0 = 0; s0 < nsteps; s0 += UNROLL) {
            static_for<0, UNROLL>([&](auto PH_) {
                const int s = s0 + decltype(PH_)::value;
                if constexpr (kWholeBlocks) {
                    step(PH_, MASK_, s);
                } else {
                    if (s < nsteps) step(PH_, MASK_, s);
                }
            });
        }
    };
    if constexpr (kWeightHalo) {
        (void)no_mask;
        if constexpr (MODE == kAdjoint) {
            if (periodic)
                run(std::integral_constant<int, 0>{});
            else
                run(std::integral_constant<int, 2>{});
        } else {
            run(std::integral_constant<int, 0>{});
        }
    } else {
        if (no_mask)
            run(std::integral_constant<int, 0>{});
        else
            run(std::integral_constant<int, 1>{});
    }
    if constexpr (MODE == kAdjoint) {
        // fold the wave's sums into its own partial row (no other wave of any
        // launch writes it concurrently; launches of one adjoint run in order)
        double *row = a.gpart + ((int64_t)blk * NW + wv) * a.npts;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            double v = gsum[t];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) row[a.npts - 1 - t] += v;
        }
    }
}

template <typename S, int DIM, int R, bool BOX, int K, int VX, int NW, int RW, int MODE = kOverlapped>
__global__ void __launch_bounds__(64 * NW)
    stream_kernel(const StreamArgs<typename ComputeOf<S>::type> a) {
    stream_tile<S, DIM, R, BOX, K, VX, NW, RW, MODE>(a, xcd_remap(blockIdx.x, a.nblocks));
}

template <typename S, int DIM, int R, int K>
__device__ void inplace_fixup_plane(const StreamArgs<typename ComputeOf<S>::type> &a, const int blk, const int zl) {
    const int64_t n0 = a.n0, n1 = a.n1, n2 = a.n2;
    int tx, ty = 0, zc;
    if constexpr (DIM == 3) {
        tx = blk % a.tiles_x;
        const int rest = blk / a.tiles_x;
        ty = rest % a.tiles_y;
        zc = rest / a.tiles_y;
    } else {
        // a 2D block holds side_nw consecutive x tiles (one per wave)
        const int groups = (a.tiles_x + a.side_nw - 1) / a.side_nw;
        tx = (blk % groups) * a.side_nw;
        zc = blk / groups;
    }
    const int z_out0 = zc * a.chunk;
    const int z_out1 = (int)(z_out0 + a.chunk < n0 ? z_out0 + a.chunk : n0);
    const int z = z_out0 + zl;
    if (z >= z_out1) return;
    const S *side = static_cast<const S *>(a.slope);
    S *dst = static_cast<S *>(a.dst);
    constexpr int KRY = DIM == 3 ? K * R : 0;
    const bool zband = zl < K * R || z >= z_out1 - K * R;
    const int zb = zl < K * R ? zl : K * R + z - (z_out1 - K * R);
    const int ntiles = DIM == 3 ? 1 : a.side_nw;  // x tiles per block in 2D
    for (int tt = 0; tt < ntiles; ++tt) {
        const int txx = tx + tt;
        if (txx >= a.tiles_x) break;
        const int64_t x0 = (int64_t)txx * a.out_x;
        const int64_t y0 = DIM == 3 ? (int64_t)ty * a.out_y : 0;
        const int ow = (int)(n2 - x0 < a.out_x ? n2 - x0 : a.out_x);
        const int oh = DIM == 3 ? (int)(n1 - y0 < a.out_y ? n1 - y0 : a.out_y) : 1;
        const int hx = a.halo_x;
        // in 2D the side blocks are per wave: block-major, wave within
        const int64_t sub = DIM == 3 ? blk : (int64_t)blk * a.side_nw + tt;
        if (zband) {
            const S *src = side + a.side_z0 + (sub * 2 * K * R + zb) * a.side_zplane;
            for (int e = threadIdx.x; e < ow * oh; e += blockDim.x) {
                const int yr = e / ow, xr = e % ow;
                dst[((int64_t)z * n1 + y0 + yr) * n2 + x0 + xr] = src[(int64_t)yr * a.out_x + xr];
            }
        } else {
            const S *src = side + (sub * a.chunk + zl) * a.side_band;
            const int nb = 2 * KRY * ow + (oh - 2 * KRY > 0 ? oh - 2 * KRY : 0) * 2 * hx;
            for (int e = threadIdx.x; e < nb; e += blockDim.x) {
                int yr, xr;
                bool ok = true;
                if (e < KRY * ow) {
                    yr = e / ow, xr = e % ow;
                    ok = yr < oh;
                } else if (e < 2 * KRY * ow) {
                    const int q = e - KRY * ow;
                    yr = oh - KRY + q / ow, xr = q % ow;
                    ok = yr >= KRY && yr >= 0;
                } else {
                    const int q = e - 2 * KRY * ow;
                    const int c = q % (2 * hx);
                    yr = KRY + q / (2 * hx);
                    xr = c < hx ? c : ow - 2 * hx + c;
                    ok = yr < oh - KRY && xr >= 0 && xr < ow && (c < hx || xr >= hx);
                }
                if (ok) dst[((int64_t)z * n1 + y0 + yr) * n2 + x0 + xr] = src[e];
            }
        }
    }
}

// Second kernel of an in-place pass: copies the band points every workgroup of
// the pass left in the side buffer into the field.  Workgroup b handles
// logical block b / kFixupParts and every kFixupParts-th output plane of it;
// the block geometry and the band index are those of the pass.
constexpr int kFixupParts = 8;
template <typename S, int DIM, int R, int K>
__global__ void __launch_bounds__(256) inplace_fixup(const StreamArgs<typename ComputeOf<S>::type> a) {
    const int blk = blockIdx.x / kFixupParts;
    for (int zl = blockIdx.x % kFixupParts; zl < a.chunk; zl += kFixupParts)
        inplace_fixup_plane<S, DIM, R, K>(a, blk, zl);
}
}  // namespace stn
