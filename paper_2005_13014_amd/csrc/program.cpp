// Batched timestep program (stencil_program_run) -- placeholder until built.
#include <hip/hip_runtime.h>

#include "../../include/stencil.h"
#include "program.hpp"

#define STENCIL_API extern "C" __attribute__((visibility("default")))

namespace stl {
int fail(int code, const char *fmt, ...);
void program_release_all() {}
}  // namespace stl

STENCIL_API int stencil_program_run(const stencil_program_t *prog, void *stream) {
    (void)prog;
    (void)stream;
    return stl::fail(STENCIL_E_UNSUPPORTED, "stencil_program_run: not available in this build");
}

STENCIL_API int stencil_hdiff_vadv_adjoint(const stencil_field_t *, const stencil_field_t *,
                                           const stencil_field_t *, const stencil_field_t *,
                                           const stencil_field_t *, const stencil_field_t *, double,
                                           const stencil_field_t *, const stencil_field_t *,
                                           const stencil_field_t *, const stencil_field_t *,
                                           const stencil_config_t *, void *) {
    return stl::fail(STENCIL_E_UNSUPPORTED, "stencil_hdiff_vadv_adjoint: not available in this build");
}
