// Kernel instantiations for mechanisms of the default reaction types
// (elementary, third-body, Lindemann, Troe) in the CONP form, the ragged
// batch kernels of those types, the LDS sizing, the fill kernel, and the
// dispatch to the CONV form (kernels_conv.hip) and to the further types'
// instantiations (kernels_ext.hip, kernels_ext_conv.hip).
#include "kernel_body.h"

namespace pj {

int64_t lds_bytes(const DevMech& dm, int mode, int S, int waves, bool grad_in_lds) {
    int64_t d = 5 * (int64_t)(dm.ns + 1);
    // Jacobian accumulator (the adjoint: only the T and V/P rows' sums), the
    // bath-gas sums; the adjoint's v and J^T v (N + 2)
    if (mode != MODE_SRC) d += (mode == MODE_ADJ ? 2 * (int64_t)dm.N : dm.nnz) + dm.ns;
    if (mode == MODE_ADJ) d += 2 * (int64_t)dm.N + 2;
    int64_t per_group = mode == MODE_ADJ && grad_in_lds ? 3 * (int64_t)dm.nr_pad : 0;
    // the sparse and dense kernels' 64 sink entries for pairs that do not exist
    if (mode == MODE_SPARSE || mode == MODE_DENSE) per_group += 64;
    return (d * S + (int64_t)RED_PER_WAVE * waves * S + per_group) * 8;
}

// zero n doubles (a kernel rather than a memset, so the call can be captured
// in a graph)
__global__ void pj_zero(double* __restrict__ p, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t zero_async(double* p, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(pj_zero, dim3(8), dim3(256), 0, stream, p, (long)n);
    return hipGetLastError();
}

hipError_t launch(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                  const double* state, const double* param, double* dstate, double* jac,
                  const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                  hipStream_t stream) {
    if (form == PJ_CONV)
        return (dm.ext ? launch_ext_conv : launch_conv)(dm, mode, form, layout, S, n, state, param, dstate, jac,
                                                        vin, grad, grad_in_lds, waves, lds, stream);
    if (dm.ext)
        return launch_ext(dm, mode, form, layout, S, n, state, param, dstate, jac, vin, grad, grad_in_lds,
                          waves, lds, stream);
    return launch_impl<false, PJ_CONP>(dm, mode, form, layout, S, n, state, param, dstate, jac, vin, grad,
                                       grad_in_lds, waves, lds, stream);
}

hipError_t launch_batch(int mode, int form, int layout, int waves, int64_t lds, const BatchSeg* d_segs,
                        int nseg, int64_t total, int ext, int su, hipStream_t stream) {
    if (ext) return launch_batch_ext(mode, form, layout, waves, lds, d_segs, nseg, total, su, stream);
    return launch_batch_impl<false>(mode, form, layout, waves, lds, d_segs, nseg, total, su, stream);
}

}  // namespace pj
