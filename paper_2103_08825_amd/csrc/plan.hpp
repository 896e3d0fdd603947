// plan.hpp -- the plan object behind the C ABI and host helpers shared by the
// C-ABI units (sweeps, batched sweeps, adjoint).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "launch.hpp"

namespace stn {

// thread-local error text; fail() records it and returns code
int fail(int code, const char *fmt, ...);
void clear_error();

#define STN_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::stn::fail(e_ == hipErrorOutOfMemory ? STENCIL_E_NOMEM : STENCIL_E_DEVICE, \
                               "%s: %s", #expr, hipGetErrorString(e_));                        \
    } while (0)

int elem_bytes(int dtype);
int enumerate_offsets(int dim, int r, int kind, int32_t *out);

// resolved execution of a plan
struct Exec {
    int method;   // STENCIL_METHOD_PLAIN / FUSED / GENERIC
    int variant;  // fused variant (0 for GENERIC)
    int k;        // steps per launch
    int chunk;    // planes per workgroup along axis 0 (0 = automatic)
};

}  // namespace stn

struct stencil_plan {
    int dim, r, kind, bc, dtype, npts;
    int64_t shape[3];
    int64_t points;
    int64_t n0, n1, n2;             // kernel view: streamed axis, y, x
    std::vector<int32_t> offsets;   // npts*dim, canonical order
    std::vector<double> coeffs;     // canonical order, as given
    std::vector<double> dense;      // (2r+1)^dim table for the fused kernels
    stencil_opts opts;
    stn::Exec exec;
    int tuned;
    // device state (bound to one device at prepare time)
    int device;
    void *scratch[2];               // [0] ping-pong field, [1] copy of an aliased input
    void *slope;                    // tessellated passes: slope rows; in-place passes: side buffer
    int64_t slope_bytes;
    int *d_off;                     // generic kernel tables
    void *d_coef;
    // recorded launches of one (d_in, d_out, T) triple (opts.graph)
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    const void *graph_in;
    void *graph_out;
    int64_t graph_T;
    int graph_failed;               // capture failed once: run with direct launches
    // adjoint: a second stream for the segment recompute and its events
    // (created on first use, on aux_device)
    hipStream_t aux_stream;
    hipEvent_t aux_ev[4];
    int aux_device;
};

namespace stn {
int plan_prepare(stencil_plan *p, hipStream_t st);
int plan_alloc_alias(stencil_plan *p);
// forget the recorded graph (the plan's execution choice or device changed)
void plan_drop_graph(stencil_plan *p);
// enqueue T steps with an explicit execution choice (no aliasing handling)
int run_passes(stencil_plan *p, const Exec &ex, const void *src, void *dst, int64_t T, hipStream_t st);
// ex with a lane width both pointers allow (falls back to the generic kernel)
Exec exec_for_ptrs(const stencil_plan *p, const void *a, const void *b);
// the same starting from `ex` instead of the plan's execution
Exec exec_for_ptrs(const stencil_plan *p, Exec ex, const void *a, const void *b);
// one step per launch (the measured plain choice where there is one)
Exec one_step_exec(const stencil_plan *p);
// launcher of one pass of k steps under ex (nullptr if none); in_place: the
// pass updates src == dst through the plan's side buffer
SweepLauncher pass_launcher(const stencil_plan *p, const Exec &ex, int k, bool in_place = false);
hipError_t launch_reduce(int dtype, const void *u, const void *ref, int64_t n, double *part,
                         double *out, hipStream_t st);
int reduce_partials_bytes();
// Stream-ordered workspace from the library's memory pool on the current
// device: up to 8 GiB of freed blocks stay reserved for later calls, so
// repeated calls do not map and unmap their workspace each time.  Free with
// hipFreeAsync.
hipError_t workspace_alloc(void **ptr, size_t bytes, hipStream_t st);
}  // namespace stn
