// Elastic (Lame) operator and GMRES(k) driver.
#include <hip/hip_runtime.h>

#include "lg_internal.h"

namespace lg {

hipError_t launch_elastic_stencil(lg_plan* p, const void* x, void* y) {
    (void)p;
    (void)x;
    (void)y;
    return hipErrorNotSupported;
}

lg_status gmres_solve(lg_plan* p, const double* b, double* x, const lg_solve_opts* o, lg_solve_info* info) {
    (void)p;
    (void)b;
    (void)x;
    (void)o;
    (void)info;
    return fail(LG_ERR_UNSUPPORTED, "elastic GMRES not built yet");
}

}  // namespace lg
