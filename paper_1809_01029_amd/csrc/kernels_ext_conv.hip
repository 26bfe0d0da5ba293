// Kernel instantiations of the CONV form for mechanisms that hold SRI
// falloff, chemically activated, P-Log or Chebyshev reactions (EXT = true).
#include "kernel_body.h"

namespace pj {

hipError_t launch_ext_conv(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                           const double* state, const double* param, double* dstate, double* jac,
                           const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                           hipStream_t stream) {
    return launch_impl<true, PJ_CONV>(dm, mode, form, layout, S, n, state, param, dstate, jac, vin, grad,
                                      grad_in_lds, waves, lds, stream);
}

}  // namespace pj
