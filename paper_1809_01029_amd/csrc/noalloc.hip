// pj_batch_eval_noalloc: the ragged batch's persistent launch without any
// device allocation.  Its segment table (the one scratch buffer of the batch
// kernels: what pj_batch_eval keeps in device memory it allocates) lives in
// a file-scope device array of NOALLOC_MAX_SEGS records, one copy per device
// for the life of the process.  Host code never passes the array's name to
// the device: the address of each device's copy is taken once per device
// with hipGetSymbolAddress and kept, and every copy and launch uses it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

// the segment table: NOALLOC_MAX_SEGS x sizeof(BatchSeg) bytes per device
static __device__ __align__(256) pj::BatchSeg scratch[pj::NOALLOC_MAX_SEGS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
pj::BatchSeg* g_ptr[MAX_DEVICES] = {};

// the device address of the current device's copy of the table, taken once
// per device (with that device current)
pj_status scratch_ptr(int dev, pj::BatchSeg** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return pj::batch_fail(PJ_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return pj::batch_fail(PJ_E_DEVICE, std::string("hipGetSymbolAddress of the segment table: ") +
                                                   hipGetErrorString(e));
        g_ptr[dev] = static_cast<pj::BatchSeg*>(p);
    }
    *out = g_ptr[dev];
    return PJ_OK;
}

}  // namespace

extern "C" pj_status pj_batch_eval_noalloc(pj_batch* b, int mode, pj_form form, pj_layout layout,
                                           pj_stream stream) {
    if (!b) return pj::batch_fail(PJ_E_INVALID, "NULL batch");
    pj_status r = pj::batch_check(b, mode, form, layout);
    if (r != PJ_OK) return r;
    if (b->segs.empty()) {
        pj::batch_ok();
        return PJ_OK;
    }
    int nseg = 0;
    for (const auto& sg : b->segs) nseg += sg.n > 0;
    if (nseg > pj::NOALLOC_MAX_SEGS)
        return pj::batch_fail(PJ_E_UNSUPPORTED, "pj_batch_eval_noalloc takes at most " +
                                                    std::to_string(pj::NOALLOC_MAX_SEGS) +
                                                    " non-empty segments, the batch has " + std::to_string(nseg));
    int S, W;
    pj::batch_shape_of(b, mode, S, W);
    if (pj::batch_lds_of(b, mode, S, W) > pj::batch_lds_limit(b))
        return pj::batch_fail(PJ_E_UNSUPPORTED, "a segment's working set exceeds the LDS of one workgroup");
    const int64_t lds = pj::batch_launch_lds(b, mode, S, W);
    const hipStream_t st = (hipStream_t)stream;
    // the adjoint's parameter sums start at zero (a fill kernel, as pj_batch_eval)
    if (mode == pj::MODE_ADJ)
        for (const auto& sg : b->segs)
            if (sg.grad) {
                hipError_t e = pj::zero_async(sg.grad, 3 * (int64_t)sg.mech->m.nr, st);
                if (e != hipSuccess)
                    return pj::batch_fail(PJ_E_DEVICE, std::string("zeroing failed: ") + hipGetErrorString(e));
            }
    if (nseg == 0) {
        pj::batch_ok();
        return PJ_OK;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return pj::batch_fail(PJ_E_DEVICE, "no HIP device");
    pj::BatchSeg* d_table = nullptr;
    r = scratch_ptr(dev, &d_table);
    if (r != PJ_OK) return r;
    // the table on the host, in the batch's own staging array
    long g0 = 0;
    int ext = 0;
    if (pj::batch_fill_table(b, mode, S, W, b->noalloc_host, pj::NOALLOC_MAX_SEGS, &g0, &ext) != nseg)
        return pj::batch_fail(PJ_E_UNSUPPORTED, "segment table does not match the batch");
    // stream-ordered: a call on the same stream waits for the previous one's
    // launch before it overwrites the table
    hipError_t e = hipMemcpyAsync(d_table, b->noalloc_host, (size_t)nseg * sizeof(pj::BatchSeg),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
        return pj::batch_fail(PJ_E_DEVICE, std::string("upload of the segment table: ") + hipGetErrorString(e));
    e = pj::launch_batch(mode, form, layout, W, lds, d_table, nseg, g0, ext,
                         pj::batch_uniform_states(b, mode, S, W), st);
    if (e != hipSuccess) return pj::batch_fail(PJ_E_DEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
    pj::batch_ok();
    return PJ_OK;
}
