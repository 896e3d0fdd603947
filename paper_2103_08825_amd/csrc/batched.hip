// batched.hip -- many independent 2D sweeps in one persistent launch.
//
// Each grid g runs P_g fused passes (k_g steps each, the last one T_g mod k_g
// steps).  A pass splits into nblk_g blocks (groups of output tiles times
// chunks of rows, exactly as a single-grid launch would).  Grids are assigned
// whole to one of kBatchParts partitions (largest work first, to the least
// loaded); each partition's work list holds its (pass, grid, block) items
// ordered by pass, then grid, then block.  The workgroups serving a partition
// take its items from the partition's atomic cursor in that order; an item of
// pass p waits until grid g's completion counter reaches p * nblk_g, i.e. until
// every block of the previous pass has been written.  An item only ever waits
// on items earlier in its partition's list, which running workgroups of that
// partition took first, so every list drains.  Every wait is bounded: a
// workgroup that spins past the limit records an error and gives up the item,
// so the kernel ends in every case.
//
// The counter reset and the persistent kernel are captured once into a HIP
// graph; stencil_batch_launch replays it.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "batched_kernel.hpp"
#include "plan.hpp"
#include "registry.hpp"
#include "variants.hpp"

struct stencil_batch {
    int device;
    int dtype;
    int64_t nitems;
    int ngrids;
    int workgroups;
    void *mem;  // one device allocation: grids, items, counters | cursors | error | bounds, scratch fields
    stn::BatchArgs args;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t wait_ticks;  // host copy of the wait limit (source of its upload)
};

namespace stn {

__global__ void batch_reset(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

static hipError_t launch_batched(int dtype, int rmax, const BatchArgs &a, int wgs, hipStream_t st) {
    switch (dtype) {
    case STENCIL_F64: return launch_batched_f64(a, rmax, wgs, st);
    case STENCIL_F32: return launch_batched_f32(a, rmax, wgs, st);
    case STENCIL_BF16: return launch_batched_bf16(a, rmax, wgs, st);
    default: return launch_batched_f16(a, rmax, wgs, st);
    }
}

static int resident_workgroups(int dtype, int rmax, int *out) {
    int dev = 0, cus = 0, per = 0;
    STN_HIP(hipGetDevice(&dev));
    STN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const void *fn = dtype == STENCIL_F64    ? batched_kernel_f64(rmax)
                     : dtype == STENCIL_F32  ? batched_kernel_f32(rmax)
                     : dtype == STENCIL_BF16 ? batched_kernel_bf16(rmax)
                                             : batched_kernel_f16(rmax);
    STN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 64 * kBatchNW, 0));
    *out = std::max(1, cus * std::max(1, per));
    return STENCIL_OK;
}

static int batch_build(stencil_batch **out, stencil_plan *const *plans, int n, const void *const *d_in,
                       void *const *d_out, const int64_t *T, int flags, hipStream_t st) {
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!plans || n < 1 || !d_in || !d_out || !T) return fail(STENCIL_E_INVALID, "bad batch arguments");
    const int dtype = plans[0] ? plans[0]->dtype : -1;
    for (int i = 0; i < n; ++i) {
        const stencil_plan *p = plans[i];
        if (!p) return fail(STENCIL_E_INVALID, "plans[%d] is NULL", i);
        if (p->dim != 2) return fail(STENCIL_E_UNSUPPORTED, "batched sweeps take 2D plans (plans[%d] is %dD)", i, p->dim);
        if (p->r > 2) return fail(STENCIL_E_UNSUPPORTED, "batched sweeps take r <= 2 (plans[%d] has r=%d)", i, p->r);
        if (p->dtype != dtype) return fail(STENCIL_E_INVALID, "plans differ in dtype");
        if (!d_in[i] || !d_out[i]) return fail(STENCIL_E_INVALID, "NULL buffer for grid %d", i);
        if (d_in[i] == d_out[i]) return fail(STENCIL_E_INVALID, "d_in[%d] aliases d_out[%d]", i, i);
        if (T[i] < 0) return fail(STENCIL_E_INVALID, "T[%d] < 0", i);
        if (p->n0 >= ((int64_t)1 << 31) || p->n2 * elem_bytes(dtype) >= ((int64_t)1 << 31))
            return fail(STENCIL_E_UNSUPPORTED, "grid %d is too large for the batched kernel", i);
    }
    if (flags & 1) {
        for (int i = 0; i < n; ++i) {
            const int rc = stencil_autotune(plans[i], st);
            if (rc != STENCIL_OK) return rc;
        }
    }
    // per-grid geometry
    std::vector<BatchGrid> grids(n);
    int max_pass = 0;
    for (int i = 0; i < n; ++i) {
        const stencil_plan *p = plans[i];
        BatchGrid &g = grids[i];
        std::memset(&g, 0, sizeof g);
        const int kmax = p->r == 1 ? kBatchMaxK1 : kBatchMaxK2;
        // plain and generic plans run one step per item; a fused plan runs its
        // requested depth, else the deepest compiled one (longer items amortise
        // the per-item fill and synchronisation; measured best on uneven batches)
        int k = kmax;
        if (p->opts.method == STENCIL_METHOD_GENERIC || p->opts.method == STENCIL_METHOD_PLAIN)
            k = 1;
        else if (p->opts.fused_k > 0)
            k = p->opts.fused_k;
        else if (flags & 1)
            k = p->exec.k;
        k = std::max(1, std::min(k, kmax));
        const int64_t Ti = T[i];
        g.k = k;
        g.krem = (int)(Ti % k);
        g.npass = (int)(Ti / k + (g.krem ? 1 : 0));
        g.in = d_in[i];
        g.out = d_out[i];
        g.n0 = p->n0;
        g.n2 = p->n2;
        g.r = p->r;
        g.box = p->kind == STENCIL_BOX ? 1 : 0;
        g.bc = p->bc;
        // an explicitly requested chunk wins; a tuned or measured single-grid chunk
        // does not carry over (it is chosen to fill the GPU with one grid)
        const int chunk = p->opts.chunk > 0 ? p->opts.chunk : kBatchChunk;
        const Geometry geo = stream_geometry(2, p->r, k, VariantShape{kBatchVX, kBatchNW, 1}, p->n0, 1, p->n2, chunk);
        if (!geo.ok) return fail(STENCIL_E_INVALID, "grid %d has no valid tiling", i);
        g.tiles_x = geo.tiles_x;
        g.chunk = geo.chunk;
        g.chunks = geo.chunks;
        g.out_x = geo.out_x;
        g.halo_x = geo.halo_x;
        g.nblk = geo.nblocks;
        const int W = 2 * p->r + 1;
        for (int q = 0; q < W * W; ++q) g.coef[q] = p->dense[q];
        max_pass = std::max(max_pass, g.npass);
    }
    // partitions: whole grids, largest work (points x T) first into the least
    // loaded partition.  (A cost model of the items' stream lengths balanced the
    // partitions' measured work better but ran 3% slower on the uneven 256-grid
    // workload: the makespan also follows the grids' chains of passes.)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto work = [&](int i) { return (double)plans[i]->points * (double)T[i]; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    std::vector<int> part_of(n, 0);
    double load[kBatchParts] = {};
    for (int i : order) {
        int best = 0;
        for (int q = 1; q < kBatchParts; ++q)
            if (load[q] < load[best]) best = q;
        part_of[i] = best;
        load[best] += work(i);
    }
    // each partition's list: pass-major; within a pass, grids with the longest
    // remaining chain of passes first (they bound the makespan)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const int64_t wx = (int64_t)grids[x].npass * grids[x].nblk, wy = (int64_t)grids[y].npass * grids[y].nblk;
        return grids[x].npass != grids[y].npass ? grids[x].npass > grids[y].npass : wx > wy;
    });
    std::vector<BatchItem> items;
    std::vector<int> part_begin(kBatchParts + 1, 0);
    for (int q = 0; q < kBatchParts; ++q) {
        part_begin[q] = (int)items.size();
        for (int pass = 0; pass < max_pass; ++pass)
            for (int i : order)
                if (part_of[i] == q && pass < grids[i].npass)
                    for (int b = 0; b < grids[i].nblk; ++b) items.push_back(BatchItem{i, pass, b, 0});
    }
    part_begin[kBatchParts] = (int)items.size();
    if (items.size() >= (size_t)0x7fffffff) return fail(STENCIL_E_UNSUPPORTED, "batch has too many work items");
    // one device allocation
    const size_t eb = elem_bytes(dtype);
    auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t grids_b = align(sizeof(BatchGrid) * n);
    const size_t items_b = align(sizeof(BatchItem) * std::max<size_t>(1, items.size()));
    // counters: per grid, then the partition cursors (one line each), the error
    // flag (the replay's reset clears these), the partition bounds and the wait
    // limit (8-byte aligned)
    const size_t ctr_ints = (size_t)n + kBatchParts * kCursorStride + 1;
    const size_t wait_off = (sizeof(int) * (ctr_ints + kBatchParts + 1) + 7) & ~(size_t)7;
    const size_t ctr_b = align(wait_off + sizeof(uint64_t));
    size_t scratch_b = 0;
    for (int i = 0; i < n; ++i)
        if (grids[i].npass > 1) scratch_b += align((size_t)plans[i]->points * eb);
    stencil_batch *b = new (std::nothrow) stencil_batch();
    if (!b) return fail(STENCIL_E_NOMEM, "out of host memory");
    b->mem = nullptr;
    b->graph = nullptr;
    b->exec = nullptr;
    b->wait_ticks = kDefaultWaitTicks;
    auto cleanup = [&](int code) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        if (b->mem) (void)hipFree(b->mem);
        delete b;
        return code;
    };
    hipError_t e = hipMalloc(&b->mem, grids_b + items_b + ctr_b + scratch_b);
    if (e != hipSuccess) {
        b->mem = nullptr;
        return cleanup(fail(STENCIL_E_NOMEM, "batch workspace: %s", hipGetErrorString(e)));
    }
    char *base = static_cast<char *>(b->mem);
    char *sc = base + grids_b + items_b + ctr_b;
    for (int i = 0; i < n; ++i)
        if (grids[i].npass > 1) {
            grids[i].scratch = sc;
            sc += align((size_t)plans[i]->points * eb);
        } else {
            grids[i].scratch = nullptr;
        }
    e = hipMemcpy(base, grids.data(), sizeof(BatchGrid) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(base + grids_b, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
    int *ctr = reinterpret_cast<int *>(base + grids_b + items_b);
    if (e == hipSuccess)
        e = hipMemcpy(ctr + ctr_ints, part_begin.data(), sizeof(int) * part_begin.size(), hipMemcpyHostToDevice);
    uint64_t *wait_dev = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(ctr) + wait_off);
    if (e == hipSuccess) e = hipMemcpy(wait_dev, &b->wait_ticks, sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(fail(STENCIL_E_DEVICE, "batch upload: %s", hipGetErrorString(e)));
    int rmax = 1;
    for (int i = 0; i < n; ++i) rmax = std::max(rmax, grids[i].r);
    int wgs = 0;
    int rc = resident_workgroups(dtype, rmax, &wgs);
    if (rc != STENCIL_OK) return cleanup(rc);
    // whole rounds of partitions (every partition needs a resident workgroup)
    if (wgs < kBatchParts) return cleanup(fail(STENCIL_E_UNSUPPORTED, "device holds too few workgroups"));
    wgs = wgs / kBatchParts * kBatchParts;
    b->dtype = dtype;
    b->ngrids = n;
    b->nitems = (int64_t)items.size();
    b->workgroups = wgs;
    b->args = BatchArgs{reinterpret_cast<const BatchGrid *>(base), reinterpret_cast<const BatchItem *>(base + grids_b),
                        ctr + ctr_ints, ctr, ctr + n, ctr + n + kBatchParts * kCursorStride, wait_dev};
    STN_HIP(hipGetDevice(&b->device));
    // capture: reset counters, cursor and error flag with a kernel, then the persistent kernel
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_reset, dim3(1), dim3(256), 0, cap, ctr, (int)ctr_ints);
        hipError_t e1 = hipGetLastError();
        // grids with T = 0 are copies
        for (int i = 0; i < n && e1 == hipSuccess; ++i)
            if (grids[i].npass == 0)
                e1 = hipMemcpyAsync(d_out[i], d_in[i], (size_t)plans[i]->points * eb, hipMemcpyDeviceToDevice, cap);
        const hipError_t e2 = launch_batched(dtype, rmax, b->args, wgs, cap);
        e = hipStreamEndCapture(cap, &b->graph);
        if (e == hipSuccess && e1 != hipSuccess) e = e1;
        if (e == hipSuccess && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return cleanup(fail(STENCIL_E_DEVICE, "batch graph capture: %s", hipGetErrorString(e)));
    *out = b;
    return STENCIL_OK;
}

}  // namespace stn

using namespace stn;

extern "C" {

int stencil_batch_create(stencil_batch **out, stencil_plan *const *plans, int n, const void *const *d_in,
                         void *const *d_out, const int64_t *T, int flags, void *stream) {
    clear_error();
    return batch_build(out, plans, n, d_in, d_out, T, flags, (hipStream_t)stream);
}

int stencil_batch_launch(stencil_batch *b, void *stream) {
    clear_error();
    if (!b) return fail(STENCIL_E_INVALID, "batch is NULL");
    int dev = 0;
    STN_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(STENCIL_E_INVALID, "batch was built on device %d", b->device);
    STN_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return STENCIL_OK;
}

void stencil_batch_destroy(stencil_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

int stencil_batch_info(const stencil_batch *b, int64_t *items, int64_t *workgroups) {
    clear_error();
    if (!b) return fail(STENCIL_E_INVALID, "batch is NULL");
    if (items) *items = b->nitems;
    if (workgroups) *workgroups = b->workgroups;
    return STENCIL_OK;
}

int stencil_batch_status(const stencil_batch *b, void *stream) {
    clear_error();
    if (!b) return fail(STENCIL_E_INVALID, "batch is NULL");
    STN_HIP(hipStreamSynchronize((hipStream_t)stream));
    int flag = 0;
    STN_HIP(hipMemcpy(&flag, b->args.error, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) return fail(STENCIL_E_DEVICE, "a batched work item waited past the spin limit");
    return STENCIL_OK;
}

int stencil_batch_set_wait_limit(stencil_batch *b, int64_t limit_us, void *stream) {
    clear_error();
    if (!b) return fail(STENCIL_E_INVALID, "batch is NULL");
    if (limit_us < 0) return fail(STENCIL_E_INVALID, "negative wait limit");
    const uint64_t cap = UINT64_MAX / kTicksPerUs;
    b->wait_ticks = (uint64_t)limit_us > cap ? UINT64_MAX : (uint64_t)limit_us * kTicksPerUs;
    // ordered after earlier replays on the stream; the host value stays in the batch
    STN_HIP(hipMemcpyAsync(const_cast<uint64_t *>(b->args.wait_ticks), &b->wait_ticks, sizeof(uint64_t),
                           hipMemcpyHostToDevice, (hipStream_t)stream));
    return STENCIL_OK;
}

int stencil_run_batched(stencil_plan *const *plans, int n, const void *const *d_in, void *const *d_out,
                        const int64_t *T, void *stream) {
    clear_error();
    stencil_batch *b = nullptr;
    int rc = batch_build(&b, plans, n, d_in, d_out, T, 0, (hipStream_t)stream);
    if (rc != STENCIL_OK) return rc;
    rc = stencil_batch_launch(b, stream);
    // the batch owns device memory the launch uses: wait before freeing it
    const int st = stencil_batch_status(b, stream);
    stencil_batch_destroy(b);
    if (rc != STENCIL_OK) return rc;
    return st;
}

}  // extern "C"
