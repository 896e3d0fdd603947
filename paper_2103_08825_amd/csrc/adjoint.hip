// adjoint.hip -- placeholder until the adjoint sweep lands.
#include "plan.hpp"
using namespace stn;
extern "C" int stencil_adjoint(stencil_plan *, const void *, const void *, int64_t, int64_t, void *, double *, void *) {
    return fail(STENCIL_E_UNSUPPORTED, "adjoint is not built yet");
}
