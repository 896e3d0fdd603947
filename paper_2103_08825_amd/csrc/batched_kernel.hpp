// batched_kernel.hpp -- the persistent kernel of the batched sweep (see batched.hip).
#pragma once

#include "stream_kernel.hpp"

namespace stn {

// the persistent kernel's tile shape: one column per lane (any width), 4 waves
constexpr int kBatchVX = 1;
constexpr int kBatchNW = 4;
// fused steps compiled for order-1 stencils: deeper items mean fewer passes and
// fewer dependency waits, which outweighs their wider recomputed halo up to 12
// (uneven 256-grid workload, 128-row items: k = 6 1004, 8 1232, 12 1376,
// 16 1181 GStencil/s; at 16 the kernel's registers leave fewer waves per CU)
constexpr int kBatchMaxK1 = 12;
constexpr int kBatchMaxK2 = 4;  // ... for order-2 stencils
// rows per work item: large enough that an item's fill (k(2r+1) extra steps) and
// bookkeeping are small, small enough that a grid's pass splits into many items
// and a long chain of passes stays short (measured on the uneven 256-grid
// workload: 128 beats 64, 256 and 512)
constexpr int kBatchChunk = 128;
// A wait gives up after a limit in ticks of the 100 MHz real-time counter
// (stencil_batch_set_wait_limit; by default about one second), or at once when
// another workgroup already gave up.
constexpr uint64_t kTicksPerUs = 100;
constexpr uint64_t kDefaultWaitTicks = 1000000ull * kTicksPerUs;

struct BatchGrid {
    const void *in;
    void *out;
    void *scratch;
    int64_t n0, n2;
    int r, box, bc, npass, k, krem, nblk;
    int tiles_x, chunk, chunks, out_x, halo_x;
    double coef[25];  // dense [dz][dx], (2r+1)^2 <= 25
};

struct BatchItem {
    int grid, pass, blk, pad;
};

// The work list is split into kBatchParts partitions, each holding whole grids;
// workgroup b serves partition b mod kBatchParts.  Workgroups are dispatched to
// the XCDs round-robin, so a partition's items (and its grids' halo re-reads)
// stay in one XCD's L2, and the partitions' cursors do not contend.
constexpr int kBatchParts = 8;
constexpr int kCursorStride = 32;  // ints between cursors: one 128-byte line each

struct BatchArgs {
    const BatchGrid *grids;
    const BatchItem *items;
    const int *part_begin;  // kBatchParts + 1 item indices
    int *counters;          // one per grid
    int *cursors;           // kBatchParts, kCursorStride apart
    int *error;
    const uint64_t *wait_ticks;  // the wait limit (not cleared between replays)
};

__device__ __forceinline__ const void *pass_src(const BatchGrid &g, int p) {
    if (p == 0) return g.in;
    return ((g.npass - p) % 2 == 0) ? g.out : g.scratch;
}
__device__ __forceinline__ void *pass_dst(const BatchGrid &g, int p) {
    return ((g.npass - (p + 1)) % 2 == 0) ? g.out : g.scratch;
}

template <typename S, int R, bool BOX, int K>
__device__ __forceinline__ void run_item(const BatchGrid &g, int pass, int blk) {
    using C = typename ComputeOf<S>::type;
    StreamArgs<C> a;
    a.src = pass_src(g, pass);
    a.dst = pass_dst(g, pass);
    a.n0 = g.n0;
    a.n1 = 1;
    a.n2 = g.n2;
    a.tiles_x = g.tiles_x;
    a.tiles_y = 1;
    a.chunks = g.chunks;
    a.chunk = g.chunk;
    a.out_x = g.out_x;
    a.out_y = 1;
    a.halo_x = g.halo_x;
    a.bc = g.bc;
    a.nblocks = g.nblk;
    constexpr int W = 2 * R + 1;
#pragma unroll
    for (int i = 0; i < W * W; ++i) a.coef[i] = (C)g.coef[i];
    stream_tile<S, 2, R, BOX, K, kBatchVX, kBatchNW, 1>(a, blk);
}

template <typename S, int R, bool BOX, int KMAX>
__device__ __forceinline__ void dispatch_k(const BatchGrid &g, int pass, int blk, int k) {
    static_for<1, KMAX + 1>([&](auto K_) {
        constexpr int K = decltype(K_)::value;
        if (k == K) run_item<S, R, BOX, K>(g, pass, blk);
    });
}

// RMAX: the largest stencil order the batch holds (1 or 2); a kernel compiled for
// order 1 only carries fewer registers, hence more waves to hide memory latency.
template <typename S, int RMAX>
__global__ void __launch_bounds__(64 * kBatchNW) batched_kernel(const BatchArgs a) {
    __shared__ int item_sh;
    __shared__ int ok_sh;
    // Within a partition, an item only waits on earlier items of the same grid,
    // which workgroups of the same partition (all resident) took first, so
    // every partition's list drains.
    //
    // Lane 0 of the workgroup does all bookkeeping in one place, between the
    // two barriers that open an iteration: it counts the item finished in the
    // previous iteration, then takes the next one.  Loop control is read back
    // with readfirstlane, so the loop is uniform for the compiler as well: two
    // separate lane-0 regions around the back-edge (count at the end, take at
    // the top) can otherwise be merged into a loop of their own that lane 0
    // enters only after the rest of its wave has left -- which it never does.
    //
    // Memory ordering.  An item of pass p > 0 reads what the items of pass p-1
    // of its grid wrote, possibly on another XCD (whose L2 is not coherent with
    // this one).  The producer's waves first wait until their own stores have
    // reached L2 (s_waitcnt 0) and meet at a barrier; lane 0 then issues one
    // agent-scope release (which writes back this XCD's L2) before counting the
    // item.  The consumer's lane 0 polls the count with relaxed loads and issues
    // one agent-scope acquire (which invalidates this compute unit's caches)
    // before the barrier that releases the other waves.  Items of a grid's last
    // pass are read by nobody (the kernel's end publishes them) and items of
    // pass 0 read only the inputs, so they skip the release and the acquire.
    int done_grid = -1;  // grid whose item (not of its last pass) finished in the previous iteration
    const int part = blockIdx.x % kBatchParts;
    const int first = a.part_begin[part], last = a.part_begin[part + 1];
    for (;;) {
        __syncthreads();  // every wave's stores of the previous item are in L2
        if (threadIdx.x == 0) {
            if (done_grid >= 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(a.counters + done_grid, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            item_sh = first + atomicAdd(a.cursors + part * kCursorStride, 1);
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(item_sh);
        if (it >= last) break;  // scalar branch: every wave leaves together
        const int grid = __builtin_amdgcn_readfirstlane(a.items[it].grid);
        const int ipass = __builtin_amdgcn_readfirstlane(a.items[it].pass);
        const int iblk = __builtin_amdgcn_readfirstlane(a.items[it].blk);
        const BatchGrid &g = a.grids[grid];
        if (threadIdx.x == 0) {
            int ok = 1;
            if (ipass > 0) {
                // poll with relaxed device-coherent loads; a single acquire follows
                const int need = ipass * g.nblk;
                const uint64_t limit = *a.wait_ticks;
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                while (__hip_atomic_load(a.counters + grid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                        __builtin_amdgcn_s_memrealtime() - t0 > limit) {
                        ok = 0;
                        __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                // the previous pass's stores (other XCDs' included) become visible
                // to every wave of this workgroup once they pass the barrier below
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            ok_sh = ok;
        }
        __syncthreads();
        const int ok = __builtin_amdgcn_readfirstlane(ok_sh);
        const int npass = __builtin_amdgcn_readfirstlane(g.npass);
        if (ok) {
            const int krem = __builtin_amdgcn_readfirstlane(g.krem);
            const int k = ipass < npass - 1 || krem == 0 ? __builtin_amdgcn_readfirstlane(g.k) : krem;
            const int r = __builtin_amdgcn_readfirstlane(g.r);
            const int box = __builtin_amdgcn_readfirstlane(g.box);
            if (r == 1) {
                if (box)
                    dispatch_k<S, 1, true, kBatchMaxK1>(g, ipass, iblk, k);
                else
                    dispatch_k<S, 1, false, kBatchMaxK1>(g, ipass, iblk, k);
            } else if constexpr (RMAX >= 2) {
                if (box)
                    dispatch_k<S, 2, true, kBatchMaxK2>(g, ipass, iblk, k);
                else
                    dispatch_k<S, 2, false, kBatchMaxK2>(g, ipass, iblk, k);
            }
        }
        if (ipass < npass - 1) {
            // this wave's stores have reached L2 before lane 0's release
            __builtin_amdgcn_s_waitcnt(0);
            done_grid = grid;
        } else {
            done_grid = -1;
        }
    }
}

// launchers and occupancy queries, one per storage type (batched_<dtype>.hip)
hipError_t launch_batched_f64(const BatchArgs &a, int rmax, int wgs, hipStream_t st);
hipError_t launch_batched_f32(const BatchArgs &a, int rmax, int wgs, hipStream_t st);
hipError_t launch_batched_bf16(const BatchArgs &a, int rmax, int wgs, hipStream_t st);
hipError_t launch_batched_f16(const BatchArgs &a, int rmax, int wgs, hipStream_t st);
const void *batched_kernel_f64(int rmax);
const void *batched_kernel_f32(int rmax);
const void *batched_kernel_bf16(int rmax);
const void *batched_kernel_f16(int rmax);

}  // namespace stn
