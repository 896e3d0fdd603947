// hip_stub.cpp -- a host-only stand-in for the HIP runtime calls the C-ABI
// layer (api.cpp, registry.cpp) makes, so its host logic can run on the CPU
// under AddressSanitizer/UndefinedBehaviorSanitizer.  Device memory is host
// memory, streams run in call order, graph capture records launches and copies
// and replays them, events read a clock that launches advance.  Kernels are
// replaced by the harness's launchers (stub_sweep), which track each buffer's
// time level in its first 8 bytes.
#include "hip_stub.h"

#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

struct ihipStream_t {
    int id;
};
struct ihipEvent_t {
    double t;
};
struct ihipGraph {
    std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
    std::vector<std::function<void()>> ops;
};

StubState g_stub;
static ihipGraph *g_recording = nullptr;  // graph being captured
static hipStream_t g_capture_stream = nullptr;

// run an operation now, or record it when its stream is being captured
void stub_enqueue(hipStream_t st, std::function<void()> op) {
    if (g_recording && st == g_capture_stream) {
        g_recording->ops.push_back(std::move(op));
        return;
    }
    op();
}

extern "C" {

hipError_t hipMalloc(void **p, size_t n) {
    if (!p) return hipErrorInvalidValue;
    *p = calloc(n ? n : 1, 1);
    g_stub.mallocs.push_back(n);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
    free(p);
    return hipSuccess;
}
hipError_t hipMallocAsync(void **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
// memory pools: one dummy pool, blocks from the host heap
hipError_t hipMemPoolCreate(hipMemPool_t *pool, const hipMemPoolProps *) {
    static int dummy;
    *pool = reinterpret_cast<hipMemPool_t>(&dummy);
    return hipSuccess;
}
hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void *) { return hipSuccess; }
hipError_t hipMemPoolDestroy(hipMemPool_t) { return hipSuccess; }
hipError_t hipMallocFromPoolAsync(void **p, size_t n, hipMemPool_t, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t st) {
    stub_enqueue(st, [=] { memmove(dst, src, n); });
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *p, int v, size_t n, hipStream_t st) {
    stub_enqueue(st, [=] { memset(p, v, n); });
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_t *prop, int) {
    memset(prop, 0, sizeof *prop);
    strcpy(prop->gcnArchName, "gfx950:sramecc+:xnack-");
    prop->multiProcessorCount = 256;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "stub error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new ihipEvent_t{0.0};
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st) {
    stub_enqueue(st, [=] { e->t = g_stub.clock_ms; });
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    *ms = (float)(b->t - a->t);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *st, unsigned int) {
    static int next = 1;
    *st = new ihipStream_t{next++};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t st) {
    delete st;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) {
    if (g_stub.capture_fails) return hipErrorStreamCaptureUnsupported;
    g_recording = new ihipGraph;
    g_capture_stream = st;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    *g = g_recording;
    g_recording = nullptr;
    g_capture_stream = nullptr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    *e = new hipGraphExec{g->ops};
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
    ++g_stub.graph_launches;
    for (auto &op : e->ops) op();
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    delete e;
    return hipSuccess;
}

}  // extern "C"
