// batched.hip -- placeholder until the persistent batched kernel lands.
#include "plan.hpp"
using namespace stn;
extern "C" {
int stencil_run_batched(stencil_plan *const *, int, const void *const *, void *const *, const int64_t *, void *) {
    return fail(STENCIL_E_UNSUPPORTED, "batched sweeps are not built yet");
}
int stencil_batch_create(stencil_batch **out, stencil_plan *const *, int, const void *const *, void *const *,
                         const int64_t *, int, void *) {
    if (out) *out = nullptr;
    return fail(STENCIL_E_UNSUPPORTED, "batched sweeps are not built yet");
}
int stencil_batch_launch(stencil_batch *, void *) { return fail(STENCIL_E_UNSUPPORTED, "not built yet"); }
void stencil_batch_destroy(stencil_batch *) {}
int stencil_batch_info(const stencil_batch *, int64_t *, int64_t *) { return fail(STENCIL_E_UNSUPPORTED, "not built yet"); }
}
