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
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batched_kernel.hpp"
#include "plan.hpp"
#include "registry.hpp"
#include "variants.hpp"

struct stencil_batch {
    int device;
    int depth[2][2];  // item depth per stencil order (1, 2) and kind (star, box); 0: none chosen
    int chunk;        // item rows chosen for grids without a requested chunk
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

// The item shape of grids whose plan requests none: depth per stencil order and
// kind (0: the deepest compiled, or the tuned single-grid depth under flags bit
// 0) and rows per item (0: kBatchChunk).
struct BatchChoice {
    int depth[2][2];
    int chunk;
};

// argument checks (host only, no device call)
static int batch_validate(stencil_plan *const *plans, int n, const void *const *d_in, void *const *d_out,
                          const int64_t *T) {
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
    return STENCIL_OK;
}

static int batch_build(stencil_batch **out, stencil_plan *const *plans, int n, const void *const *d_in,
                       void *const *d_out, const int64_t *T, int flags, hipStream_t st,
                       const BatchChoice &ch) {
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    const int vrc = batch_validate(plans, n, d_in, d_out, T);
    if (vrc != STENCIL_OK) return vrc;
    const int dtype = plans[0]->dtype;
    if (flags & 1) {
        for (int i = 0; i < n; ++i) {
            const int rc = stencil_autotune(plans[i], st);
            if (rc != STENCIL_OK) return rc;
        }
    }
    // per-grid geometry
    std::vector<BatchGrid> grids(n);
    int max_pass = 0;
    int used[2][2] = {{0, 0}, {0, 0}};  // depth taken by grids without a requested one
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
        else if (ch.depth[p->r - 1][p->kind == STENCIL_BOX ? 1 : 0] > 0)
            k = ch.depth[p->r - 1][p->kind == STENCIL_BOX ? 1 : 0];
        else if (flags & 1)
            k = p->exec.k;
        k = std::max(1, std::min(k, kmax));
        if (p->opts.method != STENCIL_METHOD_GENERIC && p->opts.method != STENCIL_METHOD_PLAIN && p->opts.fused_k <= 0)
            used[p->r - 1][p->kind == STENCIL_BOX ? 1 : 0] = k;
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
        const int chunk = p->opts.chunk > 0 ? p->opts.chunk : (ch.chunk > 0 ? ch.chunk : kBatchChunk);
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
    std::memcpy(b->depth, used, sizeof b->depth);
    b->chunk = ch.chunk > 0 ? ch.chunk : kBatchChunk;
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

// Tuning the item shape on the persistent kernel itself.  The single-grid
// tuner (flags bit 0) times launches that fill the GPU with one grid; a batch's
// items share it with thousands of others, so their best depth and row count
// differ.  Flags bit 1 instead times whole replays of the batch: a coordinate
// search over the depth of each stencil class present (order 1: 6, 8, 10, 12;
// order 2: 2, 3, 4), then over the rows per item (64 ... 256), starting from
// the defaults and keeping a candidate only if its fastest replay beats the best
// so far by more than 1%.  Candidates are built, replayed and freed in turn;
// replays read d_in and overwrite d_out only.  The choice is cached in-process
// per workload (dtype and every grid's shape, stencil, boundary, step count and
// requested options) and device architecture.

static int time_batch(stencil_batch *b, hipStream_t st, float *ms) {
    *ms = 0.f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = -1.f;
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);  // warm-up
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && (best < 0.f || t < best)) best = t;
    }
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpy(&flag, b->args.error, sizeof(int), hipMemcpyDeviceToHost);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "batch tuning replay: %s", hipGetErrorString(e));
    if (flag) return fail(STENCIL_E_DEVICE, "a batched work item waited past the spin limit while tuning");
    *ms = best;
    return STENCIL_OK;
}

static std::string batch_signature(stencil_plan *const *plans, int n, const int64_t *T) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string sig = "batch ";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        const std::string a = prop.gcnArchName;
        sig += a.substr(0, a.find(':'));
    }
    char buf[160];
    for (int i = 0; i < n; ++i) {
        const stencil_plan *p = plans[i];
        snprintf(buf, sizeof buf, "|%d %d %d %d %lld %lld %lld %d %d %d", p->dtype, p->r, p->kind, p->bc,
                 (long long)p->n0, (long long)p->n2, (long long)T[i], p->opts.method, p->opts.fused_k,
                 p->opts.chunk);
        sig += buf;
    }
    return sig;
}

// guarded by batch_tune_mutex() (batches may be created from several threads)
static std::map<std::string, BatchChoice> &batch_tune_cache() {
    static std::map<std::string, BatchChoice> m;
    return m;
}
static std::mutex &batch_tune_mutex() {
    static std::mutex m;
    return m;
}

static int batch_tune(stencil_plan *const *plans, int n, const void *const *d_in, void *const *d_out,
                      const int64_t *T, int flags, hipStream_t st, BatchChoice *best) {
    const std::string sig = batch_signature(plans, n, T);
    {
        std::lock_guard<std::mutex> g(batch_tune_mutex());
        auto it = batch_tune_cache().find(sig);
        if (it != batch_tune_cache().end()) {
            *best = it->second;
            return STENCIL_OK;
        }
    }
    // stencil classes whose depth the search may move
    bool present[2][2] = {{false, false}, {false, false}};
    for (int i = 0; i < n; ++i) {
        const stencil_plan *p = plans[i];
        if (p->opts.method == STENCIL_METHOD_GENERIC || p->opts.method == STENCIL_METHOD_PLAIN) continue;
        if (p->opts.fused_k > 0 || T[i] == 0) continue;
        present[p->r - 1][p->kind == STENCIL_BOX ? 1 : 0] = true;
    }
    BatchChoice cur{{{kBatchMaxK1, kBatchMaxK1}, {kBatchMaxK2, kBatchMaxK2}}, kBatchChunk};
    float cur_ms = 0.f;
    auto eval = [&](const BatchChoice &c, float *ms) {
        stencil_batch *b = nullptr;
        int rc = batch_build(&b, plans, n, d_in, d_out, T, flags & 1, st, c);
        if (rc == STENCIL_OK) rc = time_batch(b, st, ms);
        if (b) {
            (void)hipStreamSynchronize(st);
            stencil_batch_destroy(b);
        }
        return rc;
    };
    int rc = eval(cur, &cur_ms);
    if (rc != STENCIL_OK) return rc;
    static const int kDepths1[] = {6, 8, 10, 12};
    static const int kDepths2[] = {2, 3, 4};
    for (int r = 0; r < 2; ++r)
        for (int box = 0; box < 2; ++box) {
            if (!present[r][box]) continue;
            const int *cand = r == 0 ? kDepths1 : kDepths2;
            const int nc = r == 0 ? 4 : 3;
            for (int j = 0; j < nc; ++j) {
                if (cand[j] == cur.depth[r][box]) continue;
                BatchChoice c = cur;
                c.depth[r][box] = cand[j];
                float ms = 0.f;
                rc = eval(c, &ms);
                if (rc != STENCIL_OK) return rc;
                if (ms < 0.99f * cur_ms) {
                    cur = c;
                    cur_ms = ms;
                }
            }
        }
    static const int kRows[] = {64, 96, 128, 192, 256};
    for (int rows : kRows) {
        if (rows == cur.chunk) continue;
        BatchChoice c = cur;
        c.chunk = rows;
        float ms = 0.f;
        rc = eval(c, &ms);
        if (rc != STENCIL_OK) return rc;
        if (ms < 0.99f * cur_ms) {
            cur = c;
            cur_ms = ms;
        }
    }
    {
        std::lock_guard<std::mutex> g(batch_tune_mutex());
        batch_tune_cache()[sig] = cur;
    }
    *best = cur;
    return STENCIL_OK;
}

}  // namespace stn

using namespace stn;

extern "C" {

int stencil_batch_create(stencil_batch **out, stencil_plan *const *plans, int n, const void *const *d_in,
                         void *const *d_out, const int64_t *T, int flags, void *stream) {
    clear_error();
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (flags & ~3) return fail(STENCIL_E_INVALID, "unknown batch flags 0x%x", flags);
    BatchChoice ch{{{0, 0}, {0, 0}}, 0};
    if (flags & 2) {
        int rc = batch_validate(plans, n, d_in, d_out, T);
        if (rc != STENCIL_OK) return rc;
        rc = batch_tune(plans, n, d_in, d_out, T, flags, (hipStream_t)stream, &ch);
        if (rc != STENCIL_OK) return rc;
    }
    return batch_build(out, plans, n, d_in, d_out, T, flags & 1, (hipStream_t)stream, ch);
}

int stencil_batch_choice(const stencil_batch *b, int *depths, int *chunk) {
    clear_error();
    if (!b) return fail(STENCIL_E_INVALID, "batch is NULL");
    if (depths)
        for (int i = 0; i < 4; ++i) depths[i] = b->depth[i / 2][i % 2];
    if (chunk) *chunk = b->chunk;
    return STENCIL_OK;
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
    int rc = batch_build(&b, plans, n, d_in, d_out, T, 0, (hipStream_t)stream, BatchChoice{{{0, 0}, {0, 0}}, 0});
    if (rc != STENCIL_OK) return rc;
    rc = stencil_batch_launch(b, stream);
    // the batch owns device memory the launch uses: wait before freeing it
    const int st = stencil_batch_status(b, stream);
    stencil_batch_destroy(b);
    if (rc != STENCIL_OK) return rc;
    return st;
}

}  // extern "C"
