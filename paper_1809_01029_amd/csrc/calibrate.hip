// Calibration of the FP64 operation weights of the device's own exp, log and
// log10 (the same library routines the kernels call), for the operation
// count of the source terms' FP64 roofline: the FP64 arithmetic that one call
// executes is read off the hardware's FP64 counters over a launch of this
// kernel, minus the launch with the function left out.
#include <hip/hip_runtime.h>

#include "pjac.h"

namespace {

// out[i] = sum_{r < reps} f(in[i] + r d): one call of f, one addition and one
// multiply-add per term, so the difference to fn = 3 (no call) is the call
__global__ void pj_calibrate_kernel(int fn, long n, int reps, const double* __restrict__ in,
                                    double* __restrict__ out) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = in[i];
    double acc = 0.0;
    for (int r = 0; r < reps; ++r) {
        const double a = x + (double)r * 1.0e-3;
        acc += fn == 0 ? exp(a) : fn == 1 ? log(a) : fn == 2 ? log10(a) : a;
    }
    out[i] = acc;
}

}  // namespace

extern "C" pj_status pj_calibrate_fp64(int fn, int64_t n, int reps, const double* d_in, double* d_out,
                                       pj_stream stream) {
    if (fn < 0 || fn > 3 || n < 0 || reps < 1 || (n > 0 && (!d_in || !d_out))) return PJ_E_INVALID;
    if (n == 0) return PJ_OK;
    const int block = 256;
    const long grid = (long)((n + block - 1) / block);
    if (grid > 0x7fffffffL) return PJ_E_INVALID;
    hipLaunchKernelGGL(pj_calibrate_kernel, dim3((unsigned)grid), dim3(block), 0, (hipStream_t)stream, fn,
                       (long)n, reps, d_in, d_out);
    return hipGetLastError() == hipSuccess ? PJ_OK : PJ_E_DEVICE;
}
