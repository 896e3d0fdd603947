// adjoint.hip -- reverse-mode derivative of T stencil steps (stencil_adjoint).
//
// With lambda_T = dL/du_T, one backward step is
//     lambda_t[z] = sum_j c_j g(lambda_{t+1}, z - o_j)       (mirrored stencil)
//     dL/dc_j   += sum_x lambda_{t+1}[x] g(u_t, x + o_j)
// and dL/du_0 = lambda_0.  The mirrored stencil is the plan's own stencil with
// the weight of offset o moved to -o, run by the same sweep kernels.  Forward
// states come from checkpoints every `ckpt` steps (the fused sweep) and are
// rebuilt per segment, several steps per launch where a level-storing fused
// pass is compiled (every intermediate level stored), else one step at a time.  Where a fused adjoint pass is
// compiled for the stencil (2D and 3D, FP32 and FP64), the backward steps of a
// segment run k per launch with the coefficient sums folded into the mirrored
// sweep (stream_kernel.hpp, kAdjoint): each wave keeps FP64 sums per offset
// and adds them to its own partial row at the end of every launch.  Otherwise
// the sums run in LDS-tiled kernels (an untiled kernel covers grids with an
// axis shorter than the offsets' reach) whose workgroups keep their own FP64
// partial slots across all steps.  Either way: fixed order, no atomics, one
// fold at the end.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "device_common.hpp"
#include "plan.hpp"
#include "registry.hpp"
#include "variants.hpp"

namespace stn {

constexpr int kGradBlocks = 2048;
constexpr int kGradThreads = 256;
constexpr int kGradMaxP = 32;  // offsets per pass of the gradient kernel

// offsets of one gradient pass in the 3-axis view, uniform for every thread
struct GradOffsets {
    int ax[kGradMaxP][3];
    int reach[3];  // largest |component| per axis over the pass
};

// Untiled kernel, for grids with an axis shorter than the offsets' reach (where
// one wrap per axis is not enough): each wave takes tasks of kGradU x 64
// consecutive points of one grid row (row = (x0, x1)); lane l handles points
// c0 + l + 64 i, i < kGradU, and applies the boundary rule per point and offset.
constexpr int kGradU = 4;
constexpr int kGradTask = 64 * kGradU;

// Fold a workgroup's per-lane sums in a fixed order and add them to the
// workgroup's own slots part[block][j0 + q], q < nj.
template <int P>
__device__ __forceinline__ void fold_block(const double (&acc)[P], int j0, int nj, int npts, double *part) {
    __shared__ double sh[kGradThreads / 64][P];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        double v = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sh[w][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < nj) {
        double v = sh[0][threadIdx.x];
        for (int k = 1; k < kGradThreads / 64; ++k) v += sh[k][threadIdx.x];
        part[(int64_t)blockIdx.x * npts + j0 + threadIdx.x] += v;
    }
}

// P: accumulators compiled (8 covers the 1D-3D order-1 stars and 2D boxes; 32 the rest)
template <typename S, int P>
__global__ void __launch_bounds__(kGradThreads)
    coeff_grad_kernel(const S *__restrict__ lam, const S *__restrict__ u, int64_t n0, int64_t n1, int64_t n2,
                      int bc, const GradOffsets g, int j0, int nj, int npts, double *__restrict__ part) {
    double acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = 0.0;
    const bool periodic = bc == 1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tasks_per_row = (n2 + kGradTask - 1) / kGradTask;
    const int64_t ntask = n0 * n1 * tasks_per_row;
    const int64_t nw = (int64_t)gridDim.x * (kGradThreads / 64);
    for (int64_t tk = (int64_t)blockIdx.x * (kGradThreads / 64) + wv; tk < ntask; tk += nw) {
        const int64_t row = tk / tasks_per_row;
        const int64_t c0 = (tk - row * tasks_per_row) * kGradTask;
        const int64_t x0 = row / n1, x1 = row - x0 * n1;
#pragma unroll
        for (int i = 0; i < kGradU; ++i) {
            const int64_t x2 = c0 + lane + 64 * i;
            if (x2 >= n2) continue;
            const double l = (double)to_compute(lam[row * n2 + x2]);
#pragma unroll
            for (int q = 0; q < P; ++q) {
                int64_t y0 = x0 + g.ax[q][0], y1 = x1 + g.ax[q][1], y2 = x2 + g.ax[q][2];
                const bool inside = (y0 >= 0 && y0 < n0) && (y1 >= 0 && y1 < n1) && (y2 >= 0 && y2 < n2);
                if (!inside) {
                    y0 = wrap_index(y0, n0);
                    y1 = wrap_index(y1, n1);
                    y2 = wrap_index(y2, n2);
                }
                const double v = (double)to_compute(u[(y0 * n1 + y1) * n2 + y2]);
                acc[q] = fma(l, (inside || periodic) ? v : 0.0, acc[q]);
            }
        }
    }
    fold_block<P>(acc, j0, nj, npts, part);
}

// Tiled gradient for 2D and 3D grids.  A workgroup takes tiles of 64 rows of 64
// points (3D: 8 x 8 rows along axes 0 and 1; 2D: 64 rows along axis 0), stages
// u over the tile and its halo of RH points per axis in LDS (rows of 64 + 2 RH,
// loaded coalesced, with the boundary rule applied once per element), and
// reads lambda for its own points straight into registers.  Each lane then
// sums lambda[x] u[x + o_q] over its 16 points for every offset from LDS, so u
// is read from memory about once per tile instead of once per offset.  Tiles
// are split into 8 contiguous ranges, range x served by the workgroups that
// are dispatched to XCD x, so neighbouring tiles share their halo rows in one
// L2.
constexpr int kTileRows = 64;
constexpr int kTilePts = kTileRows / (kGradThreads / 64);  // points per lane and tile

struct TileOffsets {
    int lds[kGradMaxP];  // (o0 H1 + o1) H2 + o2 in the halo tile's layout
};

template <int T1, int RH> struct TileShape {
    static constexpr int T0 = kTileRows / T1;
    static constexpr int R0 = RH, R1 = T1 > 1 ? RH : 0, R2 = RH;
    static constexpr int H0 = T0 + 2 * R0, H1 = T1 + 2 * R1, H2 = 64 + 2 * R2;
};

// index along one axis after the boundary rule, for |y - clamp(y)| <= n: in
// range, wrapped once (periodic), or -1 (zero halo, or farther out than any
// offset reaches from a point of the grid: such elements are never used)
template <typename I> __device__ __forceinline__ I bound_index(I y, I n, bool periodic) {
    const I w = y < 0 ? y + n : (y >= n ? y - n : y);
    const bool ok = (y >= 0 && y < n) || (periodic && w >= 0 && w < n);
    return ok ? w : (I)-1;
}

// Element reads of a field as row offset + column offset.  BUF: byte offsets
// into a buffer resource of at most 2^31 - 1 bytes; an invalid row adds 2^31
// and an invalid column 2^31 - 1, so any invalid part puts the sum (no wrap
// below 2^32) past the resource's end, where the load returns 0.  Otherwise:
// 64-bit element offsets, -1 for invalid, and a select.
template <typename S, bool BUF> struct FieldReader;
template <typename S> struct FieldReader<S, true> {
    using I = int;
    using Off = uint32_t;
    rsrc_t r;
    __device__ FieldReader(const S *p, int64_t n) : r(make_rsrc(p, (uint32_t)(n * (int64_t)sizeof(S)))) {}
    static __device__ __forceinline__ Off row(I elem, bool ok) {
        return ok ? (uint32_t)elem * (uint32_t)sizeof(S) : 0x80000000u;
    }
    static __device__ __forceinline__ Off col(I elem, bool ok) {
        return ok ? (uint32_t)elem * (uint32_t)sizeof(S) : 0x7fffffffu;
    }
    __device__ __forceinline__ typename ComputeOf<S>::type get(Off row, Off col) const {
        return to_compute(__builtin_bit_cast(S, buf_load<sizeof(S)>(r, row + col)));
    }
};
template <typename S> struct FieldReader<S, false> {
    using I = int64_t;
    using Off = int64_t;
    const S *p;
    __device__ FieldReader(const S *q, int64_t) : p(q) {}
    static __device__ __forceinline__ Off row(I elem, bool ok) { return ok ? elem : (Off)-1; }
    static __device__ __forceinline__ Off col(I elem, bool ok) { return ok ? elem : (Off)-1; }
    __device__ __forceinline__ typename ComputeOf<S>::type get(Off row, Off col) const {
        using C = typename ComputeOf<S>::type;
        const bool ok = row >= 0 && col >= 0;
        const C v = to_compute(p[ok ? row + col : 0]);
        return ok ? v : (C)0;
    }
};

template <typename S, int P, int T1, int RH, bool BUF>
__global__ void __launch_bounds__(kGradThreads)
    coeff_grad_tiled(const S *__restrict__ lam, const S *__restrict__ u, int64_t n0_, int64_t n1_, int64_t n2_,
                     int bc, const TileOffsets g, int j0, int nj, int npts, double *__restrict__ part) {
    using C = typename ComputeOf<S>::type;
    using TS = TileShape<T1, RH>;
    using RD = FieldReader<S, BUF>;
    using I = typename RD::I;
    using Off = typename RD::Off;
    constexpr int T0 = TS::T0, R0 = TS::R0, R1 = TS::R1, R2 = TS::R2, H1 = TS::H1, H2 = TS::H2;
    constexpr int NROW = TS::H0 * H1;  // halo-tile rows of H2 elements
    __shared__ C tile[NROW * H2];
    // row offsets of the tile's u rows [0, NROW) and lambda rows [NROW, NROW + 64)
    __shared__ Off rowtab[NROW + kTileRows];
    static_assert(NROW + kTileRows <= kGradThreads, "one row-table entry per thread");
    double acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = 0.0;
    const bool periodic = bc == 1;
    const I n0 = (I)n0_, n1 = (I)n1_, n2 = (I)n2_, n12 = n1 * n2;
    const RD rl(lam, n0_ * n1_ * n2_), ru(u, n0_ * n1_ * n2_);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const I nt0 = (n0 + T0 - 1) / T0, nt1 = (n1 + T1 - 1) / T1, nt2 = (n2 + 63) / 64;
    const I ntile = nt0 * nt1 * nt2;
    const int xcd = blockIdx.x % 8, per = gridDim.x / 8;
    const I lo = (I)((int64_t)ntile * xcd / 8), hi = (I)((int64_t)ntile * (xcd + 1) / 8);
    // this lane's first point in the halo tile; point i (row wv + 4 i) adds
    // the constant step below
    const int base = ((R0 + (T1 > 1 ? 0 : wv)) * H1 + R1 + (T1 > 1 ? wv : 0)) * H2 + R2 + lane;
    auto step = [](int i) { return T1 > 1 ? (i >> 1) * H1 * H2 + (i & 1) * 4 * H2 : 4 * i * H2; };
    for (I tt = lo + blockIdx.x / 8; tt < hi; tt += per) {
        const I b2 = tt % nt2, b01 = tt / nt2;
        const I c0 = (b01 / nt1) * T0, c1 = (b01 % nt1) * T1, c2 = b2 * 64;
        {
            // one row-table entry per thread, axis indices after the boundary rule
            const int e = threadIdx.x;
            if (e < NROW) {
                const I y0 = bound_index<I>(c0 + e / H1 - R0, n0, periodic);
                const I y1 = bound_index<I>(c1 + e % H1 - R1, n1, periodic);
                const bool ok = y0 >= 0 && y1 >= 0;
                rowtab[e] = RD::row(ok ? y0 * n12 + y1 * n2 : 0, ok);
            } else if (e < NROW + kTileRows) {
                const int rr = e - NROW;
                const I x0 = c0 + rr / T1, x1 = c1 + rr % T1;
                const bool ok = x0 < n0 && x1 < n1;
                rowtab[e] = RD::row(ok ? x0 * n12 + x1 * n2 : 0, ok);
            }
        }
        // the table is complete, and every wave is done with the previous tile
        __syncthreads();
        // all loads of the tile issue before the first wait; invalid elements read 0
        const I x2 = c2 + lane;
        const I m2 = bound_index<I>(x2, n2, periodic);
        const Off ucol = RD::col(m2, m2 >= 0), lcol = RD::col(x2, x2 < n2);
        double l[kTilePts];
#pragma unroll
        for (int i = 0; i < kTilePts; ++i) l[i] = (double)rl.get(rowtab[NROW + wv + 4 * i], lcol);
        constexpr int NIT = (NROW + 3) / 4;
        C uv[NIT];
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int hr = k * 4 + 3 < NROW ? k * 4 + wv : min(k * 4 + wv, NROW - 1);
            uv[k] = ru.get(rowtab[hr], ucol);
        }
        // halo columns: R2 on each side of every row
        constexpr int NHALO = NROW * 2 * R2;
        constexpr int NHIT = (NHALO + kGradThreads - 1) / kGradThreads;
        C hv[NHIT];
#pragma unroll
        for (int k = 0; k < NHIT; ++k) {
            const int e0 = k * kGradThreads + (int)threadIdx.x;
            const int e = e0 < NHALO ? e0 : NHALO - 1;
            const int hr = e / (2 * R2), c = e % (2 * R2);
            const I y2 = bound_index<I>(c2 + (c < R2 ? c : 64 + c) - R2, n2, periodic);
            hv[k] = ru.get(rowtab[hr], RD::col(y2, y2 >= 0));
        }
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int hr = k * 4 + wv;
            if (hr < NROW) tile[hr * H2 + R2 + lane] = uv[k];
        }
#pragma unroll
        for (int k = 0; k < NHIT; ++k) {
            const int e = k * kGradThreads + (int)threadIdx.x;
            if (e < NHALO) {
                const int hr = e / (2 * R2), c = e % (2 * R2);
                tile[hr * H2 + (c < R2 ? c : 64 + c)] = hv[k];
            }
        }
        __syncthreads();  // the tile is complete
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (q < nj) {  // uniform
                const C *t = tile + base + g.lds[q];
#pragma unroll
                for (int i = 0; i < kTilePts; ++i) acc[q] = fma(l[i], (double)t[step(i)], acc[q]);
            }
        }
    }
    fold_block<P>(acc, j0, nj, npts, part);
}

// Tiled gradient for 1D grids: tiles of 64 x 64 consecutive points plus RH on
// each side in LDS; lane l of wave w takes points 64 (w + 4 i) + l.
template <typename S, int P, int RH, bool BUF>
__global__ void __launch_bounds__(kGradThreads)
    coeff_grad_line(const S *__restrict__ lam, const S *__restrict__ u, int64_t n_, int bc, const TileOffsets g,
                    int j0, int nj, int npts, double *__restrict__ part) {
    using C = typename ComputeOf<S>::type;
    using RD = FieldReader<S, BUF>;
    using I = typename RD::I;
    constexpr int TP = kTileRows * 64;  // points per tile
    __shared__ C tile[TP + 2 * RH];
    double acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = 0.0;
    const bool periodic = bc == 1;
    const I n = (I)n_;
    const RD rl(lam, n_), ru(u, n_);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const I ntile = (n + TP - 1) / TP;
    const int xcd = blockIdx.x % 8, per = gridDim.x / 8;
    const I lo = (I)((int64_t)ntile * xcd / 8), hi = (I)((int64_t)ntile * (xcd + 1) / 8);
    const int base = RH + 64 * wv + lane;
    for (I tt = lo + blockIdx.x / 8; tt < hi; tt += per) {
        const I c = tt * TP;
        // all loads of the tile issue before the first wait; invalid elements read 0
        double l[kTilePts];
        C uv[kTilePts];
#pragma unroll
        for (int i = 0; i < kTilePts; ++i) {
            const I x = c + base - RH + 256 * i;
            const I m = bound_index<I>(x, n, periodic);
            l[i] = (double)rl.get(RD::row(0, true), RD::col(x, x < n));
            uv[i] = ru.get(RD::row(0, true), RD::col(m, m >= 0));
        }
        C hv = (C)0;
        const int he = threadIdx.x < RH ? (int)threadIdx.x : TP + (int)threadIdx.x;  // halo slot (first 2 RH threads)
        if (threadIdx.x < 2 * RH) {
            const I y = bound_index<I>(c + he - RH, n, periodic);
            hv = ru.get(RD::row(0, true), RD::col(y, y >= 0));
        }
        __syncthreads();  // every wave is done with the previous tile
#pragma unroll
        for (int i = 0; i < kTilePts; ++i) tile[base + 256 * i] = uv[i];
        if (threadIdx.x < 2 * RH) tile[he] = hv;
        __syncthreads();  // the tile is complete
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (q < nj) {  // uniform
                const C *t = tile + base + g.lds[q];
#pragma unroll
                for (int i = 0; i < kTilePts; ++i) acc[q] = fma(l[i], (double)t[256 * i], acc[q]);
            }
        }
    }
    fold_block<P>(acc, j0, nj, npts, part);
}

// Workgroups of a gradient launch: as many as the device holds at once (a
// second, partial round would leave most compute units idle at its end), a
// multiple of 8 (one share per XCD), at most the tiles and the partial slots.
static int grad_grid(const void *kernel, int64_t ntile) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> resident;
    int dev = 0, res = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        auto it = resident.find({dev, kernel});
        if (it != resident.end()) {
            res = it->second;
        } else {
            int per = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kGradThreads, 0) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
                res = per * cus;
            resident[{dev, kernel}] = res;
        }
    }
    int64_t grid = (ntile + 7) / 8 * 8;
    if (res >= 8) grid = std::min<int64_t>(grid, res / 8 * 8);
    return (int)std::min<int64_t>(grid, kGradBlocks);
}

template <typename S, int RH>
static void launch_line(const stencil_plan *p, const S *lam, const S *u, const TileOffsets &g, int j0, int nj,
                        double *part, hipStream_t st) {
    const int64_t ntile = (p->n2 + kTileRows * 64 - 1) / (kTileRows * 64);
    const bool buf = p->points * (int64_t)sizeof(S) < ((int64_t)1 << 31);
    auto go = [&](auto kernel) {
        const int grid = grad_grid(reinterpret_cast<const void *>(kernel), ntile);
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kGradThreads), 0, st, lam, u, p->n2, p->bc, g, j0, nj, p->npts,
                           part);
    };
    buf ? go(coeff_grad_line<S, 8, RH, true>) : go(coeff_grad_line<S, 8, RH, false>);
}

template <typename S, int T1, int RH>
static void launch_tiled(const stencil_plan *p, const S *lam, const S *u, const TileOffsets &g, int j0, int nj,
                         double *part, hipStream_t st) {
    using TS = TileShape<T1, RH>;
    const int64_t ntile = ((p->n0 + TS::T0 - 1) / TS::T0) * ((p->n1 + T1 - 1) / T1) * ((p->n2 + 63) / 64);
    // 32-bit indices when every element offset (and byte offset) fits
    const bool buf = p->points * (int64_t)sizeof(S) < ((int64_t)1 << 31);
    auto go = [&](auto kernel) {
        const int grid = grad_grid(reinterpret_cast<const void *>(kernel), ntile);
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kGradThreads), 0, st, lam, u, p->n0, p->n1, p->n2, p->bc, g, j0,
                           nj, p->npts, part);
    };
    if (nj <= 8)
        buf ? go(coeff_grad_tiled<S, 8, T1, RH, true>) : go(coeff_grad_tiled<S, 8, T1, RH, false>);
    else
        buf ? go(coeff_grad_tiled<S, kGradMaxP, T1, RH, true>) : go(coeff_grad_tiled<S, kGradMaxP, T1, RH, false>);
}

// out[j] = sum over blocks of part[block][j], one workgroup per j, fixed order
__global__ void __launch_bounds__(256) coeff_grad_fold(const double *__restrict__ part, int nb, int npts,
                                                       double *__restrict__ out) {
    const int j = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[(int64_t)b * npts + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[j] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void fill_zero_f64(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

template <typename S>
static hipError_t launch_grad(const stencil_plan *p, const void *lam, const void *u, const std::vector<int> &off3,
                              double *part, hipStream_t st) {
    for (int j0 = 0; j0 < p->npts; j0 += kGradMaxP) {
        const int nj = p->npts - j0 < kGradMaxP ? p->npts - j0 : kGradMaxP;
        GradOffsets g{};  // slots past nj: offset 0 (computed, never folded)
        for (int q = 0; q < nj; ++q) {
            const int *o = &off3[3 * (j0 + q)];
            for (int i = 0; i < 3; ++i) {
                g.ax[q][i] = o[i];
                g.reach[i] = std::max(g.reach[i], std::abs(o[i]));
            }
        }
        const S *l = static_cast<const S *>(lam), *v = static_cast<const S *>(u);
        // offsets of at most 2 per axis: the LDS-tiled kernels
        const int rh = std::max(g.reach[0], std::max(g.reach[1], g.reach[2]));
        // (a single wrap per axis must reach: every axis at least as long as its reach)
        const bool fits = p->n0 >= g.reach[0] && p->n1 >= g.reach[1] && p->n2 >= g.reach[2];
        if (p->dim == 1 && rh <= 2 && fits && nj <= 8) {
            TileOffsets to{};
            for (int q = 0; q < nj; ++q) to.lds[q] = g.ax[q][2];
            rh <= 1 ? launch_line<S, 1>(p, l, v, to, j0, nj, part, st) : launch_line<S, 2>(p, l, v, to, j0, nj, part, st);
            continue;
        }
        if (p->dim >= 2 && rh <= 2 && fits) {
            TileOffsets to{};
            const bool d3 = p->dim == 3;
            const int R = rh <= 1 ? 1 : 2;
            const int H1 = d3 ? 8 + 2 * R : 1, H2 = 64 + 2 * R;
            for (int q = 0; q < nj; ++q) to.lds[q] = (g.ax[q][0] * H1 + g.ax[q][1]) * H2 + g.ax[q][2];
            if (d3)
                R == 1 ? launch_tiled<S, 8, 1>(p, l, v, to, j0, nj, part, st)
                       : launch_tiled<S, 8, 2>(p, l, v, to, j0, nj, part, st);
            else
                R == 1 ? launch_tiled<S, 1, 1>(p, l, v, to, j0, nj, part, st)
                       : launch_tiled<S, 1, 2>(p, l, v, to, j0, nj, part, st);
            continue;
        }
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3(kGradBlocks), dim3(kGradThreads), 0, st, l, v, p->n0, p->n1, p->n2, p->bc,
                               g, j0, nj, p->npts, part);
        };
        nj <= 8 ? go(coeff_grad_kernel<S, 8>) : go(coeff_grad_kernel<S, kGradMaxP>);
    }
    return hipGetLastError();
}

// one step of the stencil (weights `dense`, generic tables d_off/d_coef) from src to dst
static int one_step(stencil_plan *p, const Exec &ex, const std::vector<double> &dense, const int *d_off,
                    const void *d_coef, const void *src, void *dst, hipStream_t st) {
    const SweepLauncher fn = ex.method == STENCIL_METHOD_GENERIC ? nullptr : pass_launcher(p, ex, 1);
    if (fn) {
        SweepLaunch L{src, dst, p->n0, p->n1, p->n2, p->bc, dense.data(), ex.chunk};
        const hipError_t e = fn(L, st);
        if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "adjoint sweep launch: %s", hipGetErrorString(e));
        return STENCIL_OK;
    }
    const hipError_t e = launch_generic(p->dtype, src, dst, p->n0, p->n1, p->n2, p->npts, p->bc, d_off, d_coef, st);
    if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "adjoint generic launch: %s", hipGetErrorString(e));
    return STENCIL_OK;
}

// The fused adjoint pass (mirrored steps with the gradient folded in, kA
// steps per launch) where one is compiled for the plan's stencil: the first
// variant that has one, at its deepest compiled depth.
constexpr int kMaxAdjointK = 8;
struct FusedAdjoint {
    int variant, k;
    int chunk[kMaxAdjointK + 1];  // per depth
    int64_t rows;                 // gradient partial rows (the most any of its launches writes)
};
static bool fused_adjoint_choice(const stencil_plan *p, FusedAdjoint *out) {
    if (p->dim < 2 || (p->dtype != STENCIL_F32 && p->dtype != STENCIL_F64)) return false;
    const int box = p->kind == STENCIL_BOX ? 1 : 0;
    const int nv = p->dim == 3 ? kNumV3 : kNumV2;
    for (int v = 1; v <= nv; ++v) {
        const int k = registered_max_k(p->dtype, p->dim, p->r, box, v, 3);
        const VariantShape vs = p->dim == 3 ? kV3[v] : kV2[v];
        if (k < 1) continue;
        if (p->n1 * p->n2 * elem_bytes(p->dtype) >= ((int64_t)1 << 31) || p->n0 >= ((int64_t)1 << 31)) return false;
        if (vs.vx > 1 && p->n2 % vs.vx) continue;
        // per depth, chunks balanced over the workgroups the device holds at
        // once (the deepest pass holds about 200 registers per lane: one
        // workgroup per compute unit; shallower ones may fit more)
        FusedAdjoint fa{v, std::min(k, kMaxAdjointK), {}, 0};
        for (int kk = 1; kk <= fa.k; ++kk) {
            fa.chunk[kk] = balanced_chunk(p->dim, p->r, kk, vs, p->n0, p->n1, p->n2,
                                          resident_blocks(KernelKey{p->dtype, p->dim, p->r, box, v, kk, 3}));
            fa.rows = std::max(fa.rows, adjoint_part_rows(p->dim, p->r, kk, vs, p->n0, p->n1, p->n2, fa.chunk[kk]));
        }
        if (fa.rows <= 0) return false;
        *out = fa;
        return true;
    }
    return false;
}

constexpr int kMaxLevelsK = 8;  // deepest level-storing pass the recompute uses

// The plan's second stream and its events for the adjoint's overlapped
// recompute, created on first use on the current device (default priority).
static int aux_stream_ready(stencil_plan *p) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return STENCIL_E_DEVICE;
    if (p->aux_stream && p->aux_device == dev) return STENCIL_OK;
    for (hipEvent_t &e : p->aux_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
    p->aux_stream = nullptr;
    bool ok = hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t &e : p->aux_ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (hipEvent_t &e : p->aux_ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
        p->aux_stream = nullptr;
        (void)hipGetLastError();  // the sequential path runs instead; keep no error behind
        return STENCIL_E_DEVICE;
    }
    p->aux_device = dev;
    return STENCIL_OK;
}

// The level-storing forward pass for a segment's recompute, where one is
// compiled: (variant, deepest k) and, per depth, the chunk balanced over the
// workgroups the device holds at once; k = 0 when none.
static void levels_choice(const stencil_plan *p, int *variant, int *k, int (&chunk)[kMaxLevelsK + 1]) {
    *variant = 0;
    *k = 0;
    for (int &c : chunk) c = 0;
    if (p->dim < 2) return;
    const int box = p->kind == STENCIL_BOX ? 1 : 0;
    const int nv = p->dim == 3 ? kNumV3 : kNumV2;
    for (int v = 1; v <= nv; ++v) {
        const int kk = registered_max_k(p->dtype, p->dim, p->r, box, v, 4);
        const VariantShape vs = p->dim == 3 ? kV3[v] : kV2[v];
        if (kk < 2 || (vs.vx > 1 && p->n2 % vs.vx)) continue;
        if (p->n1 * p->n2 * elem_bytes(p->dtype) >= ((int64_t)1 << 31) || p->n0 >= ((int64_t)1 << 31)) return;
        *variant = v;
        *k = std::min(kk, kMaxLevelsK);
        for (int j = 2; j <= *k; ++j)
            chunk[j] = balanced_chunk(p->dim, p->r, j, vs, p->n0, p->n1, p->n2,
                                      resident_blocks(KernelKey{p->dtype, p->dim, p->r, box, v, j, 4}));
        return;
    }
}

static int adjoint_impl(stencil_plan *p, const Exec &ex, const Exec &ex1, const void *d_u0, const void *d_gT, int64_t T,
                        int64_t C, void *d_gu, double *d_gc, hipStream_t st) {
    const size_t field = (size_t)p->points * elem_bytes(p->dtype);
    if (T == 0) {
        if (d_gu != d_gT) STN_HIP(hipMemcpyAsync(d_gu, d_gT, field, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(fill_zero_f64, dim3(1), dim3(64), 0, st, d_gc, (int64_t)p->npts);
        STN_HIP(hipGetLastError());
        return STENCIL_OK;
    }
    const int64_t nseg = (T + C - 1) / C;
    const int64_t seglen = T < C ? T : C;
    // mirrored weights: offset o takes the weight of -o (the dense table reversed)
    std::vector<double> dense_m(p->dense.rbegin(), p->dense.rend());
    // mirrored generic tables (offsets negated, weights unchanged)
    std::vector<int> off3(3 * p->npts, 0), off3m(3 * p->npts, 0);
    static const int view_axis[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 1, 2}};
    for (int j = 0; j < p->npts; ++j)
        for (int i = 0; i < p->dim; ++i) {
            off3[3 * j + view_axis[p->dim][i]] = p->offsets[j * p->dim + i];
            off3m[3 * j + view_axis[p->dim][i]] = -p->offsets[j * p->dim + i];
        }
    // workspace (stream ordered): checkpoints 1..nseg-1, segment states 1..seglen-1,
    // two adjoint fields, partial sums, offset tables
    // every sub-buffer starts on a 256-byte boundary (the lane width chosen from
    // the caller's pointers assumes workspace fields at least as aligned)
    const int64_t nck = nseg - 1, nst = seglen - 1;
    const size_t fstride = (field + 255) & ~(size_t)255;
    FusedAdjoint fa{0, 0, {}, 0};
    const bool fused = fused_adjoint_choice(p, &fa);
    // The fused path rebuilds segment s-1 on a second stream while the mirrored
    // steps of segment s run: two segment buffers, used alternately.
    const bool overlap = fused && nseg > 1 && nst > 0 && aux_stream_ready(p) == STENCIL_OK;
    const int64_t nbuf = overlap ? 2 : 1;
    const int64_t prow = fused ? fa.rows : kGradBlocks;  // partial rows of npts doubles
    const size_t part_bytes = (size_t)prow * p->npts * sizeof(double);
    const size_t tab_bytes = off3m.size() * sizeof(int);
    const size_t ws_bytes = (size_t)(nck + nbuf * nst + 2) * fstride + part_bytes + tab_bytes;
    char *ws = nullptr;
    STN_HIP(workspace_alloc((void **)&ws, ws_bytes, st));
    auto ck = [&](int64_t s) -> void * { return s == 0 ? const_cast<void *>(d_u0) : ws + (size_t)(s - 1) * fstride; };
    char *seg_buf[2] = {ws + (size_t)nck * fstride, ws + (size_t)(nck + (nbuf - 1) * nst) * fstride};
    char *lam_buf[2] = {ws + (size_t)(nck + nbuf * nst) * fstride, ws + (size_t)(nck + nbuf * nst + 1) * fstride};
    double *part = reinterpret_cast<double *>(ws + (size_t)(nck + nbuf * nst + 2) * fstride);
    int *d_offm = reinterpret_cast<int *>(reinterpret_cast<char *>(part) + part_bytes);
    hipStream_t st2 = overlap ? p->aux_stream : st;
    hipEvent_t ev_fwd = overlap ? p->aux_ev[0] : nullptr, ev_rec = overlap ? p->aux_ev[1] : nullptr;
    hipEvent_t ev_adj = overlap ? p->aux_ev[2] : nullptr, ev_tail = overlap ? p->aux_ev[3] : nullptr;
#define STN_HIP_DONE(expr)                                                                          \
    do {                                                                                            \
        const hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return done(fail(STENCIL_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    int rc = STENCIL_OK;
    auto done = [&](int code) {
        if (overlap) {
            // nothing on the second stream may outlive the workspace
            (void)hipEventRecord(ev_tail, st2);
            (void)hipStreamWaitEvent(st, ev_tail, 0);
        }
        (void)hipFreeAsync(ws, st);
        return code;
    };
    hipError_t e = hipMemcpyAsync(d_offm, off3m.data(), off3m.size() * sizeof(int), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return done(fail(STENCIL_E_DEVICE, "adjoint table upload: %s", hipGetErrorString(e)));
    hipLaunchKernelGGL(fill_zero_f64, dim3(256), dim3(256), 0, st, part, prow * p->npts);

    // forward: checkpoints u_{s C}
    for (int64_t s = 1; s < nseg && rc == STENCIL_OK; ++s) rc = run_passes(p, ex, ck(s - 1), ck(s), C, st);
    if (rc != STENCIL_OK) return done(rc);

    int lvar = 0, lk = 0, lchunk[kMaxLevelsK + 1];
    levels_choice(p, &lvar, &lk, lchunk);
    // forward state t of segment s (t in [tb, te)): the checkpoint, else the
    // segment buffer the segment was rebuilt into
    auto seg_state = [&](int64_t s, int64_t t) -> const void * {
        const int64_t tb = s * C;
        return t == tb ? ck(s) : static_cast<const void *>(seg_buf[s & 1] + (size_t)(t - tb - 1) * fstride);
    };
    // rebuild states tb+1 .. te-1 of segment s on stream `sq`
    auto recompute = [&](int64_t s, hipStream_t sq) -> int {
        const int64_t tb = s * C, te = (tb + C < T) ? tb + C : T;
        for (int64_t t = tb + 1; t < te;) {
            const int kk = (int)std::min<int64_t>(lk, te - t);
            if (kk >= 2) {
                // states t .. t+kk-1 in one launch: level j to state(t-1+j)
                SweepLaunch L{seg_state(s, t - 1), const_cast<void *>(seg_state(s, t + kk - 1)), p->n0, p->n1, p->n2,
                              p->bc, p->dense.data(), lchunk[kk], nullptr, {}, nullptr};
                for (int j = 1; j < kk; ++j) L.ustate[j - 1] = seg_state(s, t - 1 + j);
                const SweepLauncher fn =
                    find_launcher(KernelKey{p->dtype, p->dim, p->r, p->kind == STENCIL_BOX ? 1 : 0, lvar, kk, 4});
                if (!fn) return fail(STENCIL_E_UNSUPPORTED, "no level-storing kernel with k=%d", kk);
                const hipError_t le = fn(L, sq);
                if (le != hipSuccess) return fail(STENCIL_E_DEVICE, "recompute launch: %s", hipGetErrorString(le));
                t += kk;
            } else {
                const int r1 = one_step(p, ex1, p->dense, p->d_off, p->d_coef, seg_state(s, t - 1),
                                        const_cast<void *>(seg_state(s, t)), sq);
                if (r1 != STENCIL_OK) return r1;
                ++t;
            }
        }
        return STENCIL_OK;
    };
    if (overlap) STN_HIP_DONE(hipEventRecord(ev_fwd, st));

    const void *lam = d_gT;
    int flip = 0;
    for (int64_t s = nseg - 1; s >= 0; --s) {
        const int64_t tb = s * C, te = (tb + C < T) ? tb + C : T;
        auto state = [&](int64_t t) -> const void * { return seg_state(s, t); };
        if (!overlap) {
            rc = recompute(s, st);
        } else {
            // segment s: rebuilt on this stream (the last one) or on the second
            // stream during the previous iteration
            if (s == nseg - 1)
                rc = recompute(s, st);
            else
                STN_HIP_DONE(hipStreamWaitEvent(st, ev_rec, 0));
            // segment s-1 on the second stream, into the buffer the mirrored steps
            // of segment s+1 have finished reading (the first time: after the
            // forward sweep wrote the checkpoints)
            if (rc == STENCIL_OK && s >= 1) {
                STN_HIP_DONE(hipStreamWaitEvent(st2, s == nseg - 1 ? ev_fwd : ev_adj, 0));
                rc = recompute(s - 1, st2);
                if (rc == STENCIL_OK) STN_HIP_DONE(hipEventRecord(ev_rec, st2));
            }
        }
        if (rc != STENCIL_OK) return done(rc);
        if (fused) {
            // kA mirrored steps per launch, each level pairing with its forward state
            for (int64_t t = te - 1; t >= tb;) {
                const int kk = (int)std::min<int64_t>(fa.k, t - tb + 1);
                void *out = (t + 1 - kk == 0) ? d_gu : lam_buf[flip];
                SweepLaunch L{lam, out, p->n0, p->n1, p->n2, p->bc, dense_m.data(), fa.chunk[kk], nullptr, {}, part};
                for (int j = 1; j <= kk; ++j) L.ustate[j - 1] = state(t + 1 - j);
                const SweepLauncher fn =
                    find_launcher(KernelKey{p->dtype, p->dim, p->r, p->kind == STENCIL_BOX ? 1 : 0, fa.variant, kk, 3});
                if (!fn) return done(fail(STENCIL_E_UNSUPPORTED, "no fused adjoint kernel with k=%d", kk));
                e = fn(L, st);
                if (e != hipSuccess) return done(fail(STENCIL_E_DEVICE, "adjoint launch: %s", hipGetErrorString(e)));
                lam = out;
                flip ^= 1;
                t -= kk;
            }
            if (overlap) STN_HIP_DONE(hipEventRecord(ev_adj, st));
            continue;
        }
        for (int64_t t = te - 1; t >= tb; --t) {
            e = p->dtype == STENCIL_F64 ? launch_grad<double>(p, lam, state(t), off3, part, st)
                                        : launch_grad<float>(p, lam, state(t), off3, part, st);
            if (e != hipSuccess) return done(fail(STENCIL_E_DEVICE, "gradient launch: %s", hipGetErrorString(e)));
            void *out = (t == 0) ? d_gu : lam_buf[flip];
            // the generic fallback needs mirrored weights in compute precision on the device:
            // the plan's d_coef holds the weights in canonical order, which pair with d_offm
            rc = one_step(p, ex1, dense_m, d_offm, p->d_coef, lam, out, st);
            if (rc != STENCIL_OK) return done(rc);
            lam = out;
            flip ^= 1;
        }
    }
    hipLaunchKernelGGL(coeff_grad_fold, dim3(p->npts), dim3(256), 0, st, (const double *)part, (int)prow, p->npts,
                       d_gc);
    e = hipGetLastError();
    if (e != hipSuccess) return done(fail(STENCIL_E_DEVICE, "gradient fold: %s", hipGetErrorString(e)));
    return done(STENCIL_OK);
}
#undef STN_HIP_DONE

}  // namespace stn

using namespace stn;

extern "C" int stencil_adjoint(stencil_plan *p, const void *d_u0, const void *d_gT, int64_t T,
                               int64_t checkpoint_every, void *d_grad_u0, double *d_grad_coeffs, void *stream) {
    clear_error();
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (!d_u0 || !d_gT || !d_grad_u0 || !d_grad_coeffs) return fail(STENCIL_E_INVALID, "NULL pointer");
    if (T < 0) return fail(STENCIL_E_INVALID, "T must be >= 0");
    if (checkpoint_every < 1) return fail(STENCIL_E_INVALID, "checkpoint_every must be >= 1");
    if (p->dtype != STENCIL_F64 && p->dtype != STENCIL_F32)
        return fail(STENCIL_E_UNSUPPORTED, "the adjoint supports FP64 and FP32 plans");
    if (d_grad_u0 == d_u0 || (d_grad_u0 == d_gT && T > 0))
        return fail(STENCIL_E_INVALID, "d_grad_u0 must not alias d_u0 or d_gT");
    hipStream_t st = (hipStream_t)stream;
    const int rc = plan_prepare(p, st);
    if (rc != STENCIL_OK) return rc;
    // the workspace is 256-byte aligned; the caller's three buffers decide the lane
    // width (alignments are powers of two, so OR-ing two addresses keeps the weaker)
    const void *either = reinterpret_cast<const void *>((uintptr_t)d_u0 | (uintptr_t)d_gT);
    const Exec ex = exec_for_ptrs(p, either, d_grad_u0);                     // checkpoint passes
    const Exec ex1 = exec_for_ptrs(p, one_step_exec(p), either, d_grad_u0);  // single steps
    return adjoint_impl(p, ex, ex1, d_u0, d_gT, T, checkpoint_every, d_grad_u0, d_grad_coeffs, st);
}
