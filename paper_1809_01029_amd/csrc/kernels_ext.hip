// Kernel instantiations for mechanisms that hold SRI falloff, chemically
// activated, P-Log or Chebyshev reactions (EXT = true): the CONP form and the
// ragged batch kernels.
#include "kernel_body.h"

namespace pj {

hipError_t launch_ext(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                      const double* state, const double* param, double* dstate, double* jac,
                      const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                      hipStream_t stream) {
    return launch_impl<true, PJ_CONP>(dm, mode, form, layout, S, n, state, param, dstate, jac, vin, grad,
                                      grad_in_lds, waves, lds, stream);
}

hipError_t launch_batch_ext(int mode, int form, int layout, int waves, int64_t lds, const BatchSeg* d_segs,
                            int nseg, int64_t total, int su, hipStream_t stream) {
    return launch_batch_impl<true>(mode, form, layout, waves, lds, d_segs, nseg, total, su, stream);
}

}  // namespace pj
