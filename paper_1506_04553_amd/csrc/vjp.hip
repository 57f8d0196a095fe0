// vjp.hip -- adjoint of the long-range force and potential.
#include "internal.h"

namespace p3t {

int launch_vjp(p3t_ctx *ctx, const double *, const double *, double *, double *) {
    return set_error(ctx, P3T_EINVAL, "VJP not available in this build");
}

}  // namespace p3t
