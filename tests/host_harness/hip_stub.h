// hip_stub.h -- state of the host-only HIP stand-in shared with the harness.
#pragma once

#include <hip/hip_runtime_api.h>

#include <functional>
#include <vector>

struct StubState {
    double clock_ms = 0.0;        // advanced by the stub launchers
    bool capture_fails = false;   // hipStreamBeginCapture refuses
    int graph_launches = 0;
    std::vector<size_t> mallocs;  // sizes of every hipMalloc
};
extern StubState g_stub;

void stub_enqueue(hipStream_t st, std::function<void()> op);
