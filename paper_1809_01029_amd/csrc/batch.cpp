// C-ABI of ragged multi-mechanism batches (declared in include/pjac.h):
// segments of states of different mechanisms evaluated by one persistent
// launch (or, per mode, by one launch per segment at each mechanism's own
// launch shape), optionally captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace {

thread_local std::string g_err;

pj_status fail(pj_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

bool batch_mode(int mode) { return mode == pj::MODE_SRC || mode == pj::MODE_SPARSE || mode == pj::MODE_ADJ; }

// the most states per group of a batch's launch shape (and of any segment)
int batch_cap(int mode) { return mode == pj::MODE_ADJ ? pj::MAX_S_ADJ : pj::BATCH_MAX_S; }

}  // namespace


namespace {

int64_t seg_lds(const pj_batch::Seg& sg, int mode, int S, int W) {
    return pj::lds_bytes(sg.mech->m.dm, mode, S, W, false);
}

int lds_max_of(const pj_batch* b) { return b->segs.empty() ? 0 : b->segs[0].mech->m.lds_max; }

// bytes of the adjoint's per-reaction parameter sums of one segment in LDS
int64_t seg_gr(const pj_batch::Seg& sg) { return 3 * (int64_t)sg.mech->m.dm.nr_pad * 8; }

// The persistent launch of a batch at shape S x W for a mode.  The adjoint
// keeps each segment's parameter sums in LDS after its states' arrays when
// every segment's fit at S states (else they go to the output per group).
// need: the largest LDS a segment takes at S states; the workgroups a
// compute unit then holds, k = LDS / need, set the budget LDS / k, and each
// segment takes the most states per group (S doubled, at most BATCH_MAX_S,
// the adjoint MAX_S_ADJ) whose LDS fits it: the largest mechanism keeps S,
// smaller ones hold more states at the same occupancy.  lds: the launch's
// LDS per workgroup (the largest segment's at its states).
struct Plan {
    int mode = 0, S = 1, W = 1;
    bool gr = false;
    int64_t need = 0, budget = 0;

    int64_t tot(const pj_batch::Seg& sg, int s) const { return seg_lds(sg, mode, s, W) + (gr ? seg_gr(sg) : 0); }
    // states per group of a segment
    int states(const pj_batch::Seg& sg) const {
        int s = S;
        if (sg.n > 0)
            while (s * 2 <= batch_cap(mode) && tot(sg, s * 2) <= budget) s *= 2;
        return s;
    }
    // LDS offset (doubles) of a segment's parameter sums, or -1
    int64_t gr_off(const pj_batch::Seg& sg) const { return gr ? seg_lds(sg, mode, states(sg), W) / 8 : -1; }
};

Plan make_plan(const pj_batch* b, int mode, int S, int W) {
    Plan pl;
    pl.mode = mode;
    pl.S = S;
    pl.W = W;
    const int64_t mx = lds_max_of(b);
    auto need = [&]() {
        int64_t l = 0;
        for (auto& sg : b->segs)
            if (sg.n > 0) l = std::max(l, pl.tot(sg, S));
        return l;
    };
    pl.gr = mode == pj::MODE_ADJ;
    if (pl.gr && need() > mx) pl.gr = false;
    pl.need = need();
    const int64_t k = pl.need > 0 ? std::max<int64_t>(1, mx / pl.need) : 1;
    pl.budget = std::max(pl.need, mx / k);
    return pl;
}

// the launch's LDS per workgroup: the largest segment's at its states
int64_t plan_lds(const pj_batch* b, const Plan& pl) {
    int64_t l = 0;
    for (auto& sg : b->segs)
        if (sg.n > 0) l = std::max(l, pl.tot(sg, pl.states(sg)));
    return l;
}

// the LDS the batch needs at S x W (its largest segment at S states)
int64_t batch_lds(const pj_batch* b, int mode, int S, int W) { return make_plan(b, mode, S, W).need; }

// the states per group shared by every non-empty segment, when 1, 2 or 4
int uniform_states(const pj_batch* b, int mode, int S, int W) {
    const Plan pl = make_plan(b, mode, S, W);
    int u = 0;
    for (auto& sg : b->segs) {
        if (sg.n == 0) continue;
        const int s = pl.states(sg);
        if (u && s != u) return 0;
        u = s;
    }
    return u == 1 || u == 2 || u == 4 ? u : 0;
}

// launch shape of the batch for a mode: the user's (or autotuned) if it
// fits, else the most states per workgroup (<= 4) that fit every segment's
// working set, with enough waves for about 8 resident waves per compute unit
void batch_shape(const pj_batch* b, int mode, int& S, int& W) {
    const int mx = lds_max_of(b);
    S = 1;
    for (int c = 4; c >= 1; c >>= 1)
        if (batch_lds(b, mode, c, 1) <= mx) { S = c; break; }
    if (b->user_S[mode] && b->user_S[mode] <= batch_cap(mode) &&
        batch_lds(b, mode, b->user_S[mode], b->user_W[mode] ? b->user_W[mode] : 1) <= mx)
        S = b->user_S[mode];
    W = 1;
    while (W < 8) {
        const int64_t l = batch_lds(b, mode, S, W);
        if (l > mx || (mx / l) * W >= 8) break;
        W *= 2;
    }
    if (b->user_W[mode] && batch_lds(b, mode, S, b->user_W[mode]) <= mx) W = b->user_W[mode];
}

pj_status check_segments(const pj_batch* b, int mode, pj_form form, pj_layout layout) {
    if (!batch_mode(mode)) return fail(PJ_E_INVALID, "batch mode must be 0 (source), 1 (sparse) or 3 (adjoint)");
    if (form != PJ_CONP && form != PJ_CONV) return fail(PJ_E_INVALID, "bad form");
    if (layout != PJ_LAYOUT_F && layout != PJ_LAYOUT_C) return fail(PJ_E_INVALID, "bad layout");
    int dev = -1;
    for (size_t i = 0; i < b->segs.size(); ++i) {
        const auto& sg = b->segs[i];
        const std::string at = "segment " + std::to_string(i) + ": ";
        if (!sg.mech->m.dbuf) return fail(PJ_E_INVALID, at + "mechanism not uploaded to a device");
        if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(PJ_E_DEVICE, "no HIP device");
        if (sg.mech->m.device != dev)
            return fail(PJ_E_INVALID, at + "the current HIP device is not the one the mechanism was loaded on");
        if (sg.n == 0) continue;
        if (!sg.state || !sg.param) return fail(PJ_E_INVALID, at + "NULL state or parameter");
        if (mode == pj::MODE_SRC && !sg.dstate) return fail(PJ_E_INVALID, at + "NULL source-term output");
        if (mode != pj::MODE_SRC && !sg.out) return fail(PJ_E_INVALID, at + "NULL output");
        if (mode == pj::MODE_ADJ && !sg.v) return fail(PJ_E_INVALID, at + "NULL vector v");
    }
    return PJ_OK;
}

// (re)build the device segment table for the shape S x W of a mode
// The persistent launch's segment table at S x W (the non-empty segments in
// order) into t (room for cap entries): the number of entries, or -1 if they
// exceed cap; *total: the groups of all, *ext: some segment's mechanism holds
// the further reaction types.
int fill_table(const pj_batch* b, int mode, int S, int W, pj::BatchSeg* t, int cap, long* total, int* ext) {
    const Plan pl = make_plan(b, mode, S, W);
    long g0 = 0;
    int k = 0;
    *ext = 0;
    for (auto& sg : b->segs) {
        if (sg.n == 0) continue;
        if (k >= cap) return -1;
        const int s = pl.states(sg);
        pj::BatchSeg& x = t[k++];
        x = pj::BatchSeg{};
        x.dm = sg.mech->m.dm;
        x.n = (long)sg.n;
        x.state = pj::gptr(sg.state);
        x.param = pj::gptr(sg.param);
        x.dstate = pj::gptr(sg.dstate);
        x.out = pj::gptr(sg.out);
        x.vin = pj::gptr(sg.v);
        x.grad = pj::gptr(sg.grad);
        x.g0 = g0;
        x.S = s;
        x.gr_off = pl.gr_off(sg);
        g0 += (long)((sg.n + s - 1) / s);
        *ext |= sg.mech->m.dm.ext;
    }
    *total = g0;
    return k;
}

pj_status upload_table(pj_batch* b, int mode, int S, int W) {
    if (b->table_valid && b->table_S == S && b->table_W == W && b->table_mode == mode) return PJ_OK;
    std::vector<pj::BatchSeg> t(b->segs.size());
    long g0 = 0;
    int ext = 0;
    t.resize((size_t)fill_table(b, mode, S, W, t.data(), (int)t.size(), &g0, &ext));
    const size_t bytes = std::max<size_t>(1, t.size()) * sizeof(pj::BatchSeg);
    if (bytes > b->d_cap) {
        if (b->d_segs) (void)hipFree(b->d_segs);
        b->d_segs = nullptr;
        b->d_cap = 0;
        if (hipMalloc(&b->d_segs, bytes) != hipSuccess) return fail(PJ_E_DEVICE, "hipMalloc of the segment table failed");
        b->d_cap = bytes;
    }
    if (!t.empty() && hipMemcpy(b->d_segs, t.data(), t.size() * sizeof(pj::BatchSeg), hipMemcpyHostToDevice) != hipSuccess)
        return fail(PJ_E_DEVICE, "upload of the segment table failed");
    b->table_S = S;
    b->table_W = W;
    b->table_mode = mode;
    b->table_nseg = (int)t.size();
    b->table_total = g0;
    b->table_valid = true;
    return PJ_OK;
}

// enqueue the whole batch (zeroing of the adjoint sums, then one launch)
pj_status enqueue(pj_batch* b, int mode, pj_form form, pj_layout layout, int S, int W, hipStream_t st) {
    pj_status r = upload_table(b, mode, S, W);
    if (r != PJ_OK) return r;
    if (mode == pj::MODE_ADJ)
        for (auto& sg : b->segs)
            if (sg.grad) {
                hipError_t e = pj::zero_async(sg.grad, 3 * (int64_t)sg.mech->m.nr, st);
                if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("zeroing failed: ") + hipGetErrorString(e));
            }
    if (b->table_total == 0) return PJ_OK;
    const int64_t lds = plan_lds(b, make_plan(b, mode, S, W));
    int ext = 0;   // the further reaction types' kernels if any segment needs them
    for (auto& sg : b->segs) ext |= sg.mech->m.dm.ext;
    hipError_t e = pj::launch_batch(mode, form, layout, W, lds, b->d_segs, b->table_nseg, b->table_total, ext,
                                    uniform_states(b, mode, S, W), st);
    if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
    return PJ_OK;
}

// one launch per segment, each at its mechanism's launch shape for the mode
// (the single-mechanism entry points, which also clear the adjoint's sums)
pj_status enqueue_segments(pj_batch* b, int mode, pj_form form, pj_layout layout, hipStream_t st) {
    for (size_t i = 0; i < b->segs.size(); ++i) {
        const auto& sg = b->segs[i];
        pj_status r;
        if (mode == pj::MODE_SRC)
            r = pj_eval_source(sg.mech, form, layout, sg.n, sg.state, sg.param, sg.dstate, st);
        else if (mode == pj::MODE_SPARSE)
            r = pj_eval_jacobian_sparse(sg.mech, form, layout, sg.n, sg.state, sg.param, sg.out, sg.dstate, st);
        else
            r = pj_eval_adjoint(sg.mech, form, layout, sg.n, sg.state, sg.param, sg.v, sg.out, sg.grad, sg.dstate, st);
        if (r != PJ_OK) return fail(r, "segment " + std::to_string(i) + ": " + pj_last_error());
    }
    return PJ_OK;
}

// the batch as configured for the mode: one persistent launch of shape S x W,
// or one launch per segment
pj_status enqueue_mode(pj_batch* b, int mode, pj_form form, pj_layout layout, int S, int W, hipStream_t st) {
    return b->per_seg[mode] ? enqueue_segments(b, mode, form, layout, st) : enqueue(b, mode, form, layout, S, W, st);
}

}  // namespace

// the batch internals the allocation-free entry point (noalloc.hip) shares
namespace pj {
pj_status batch_fail(pj_status st, const std::string& msg) { return fail(st, msg); }
void batch_ok() { g_err.clear(); }
pj_status batch_check(const pj_batch* b, int mode, pj_form form, pj_layout layout) {
    return check_segments(b, mode, form, layout);
}
void batch_shape_of(const pj_batch* b, int mode, int& S, int& W) { batch_shape(b, mode, S, W); }
int64_t batch_lds_of(const pj_batch* b, int mode, int S, int W) { return batch_lds(b, mode, S, W); }
int64_t batch_launch_lds(const pj_batch* b, int mode, int S, int W) {
    return plan_lds(b, make_plan(b, mode, S, W));
}
int batch_fill_table(const pj_batch* b, int mode, int S, int W, BatchSeg* t, int cap, long* total, int* ext) {
    return fill_table(b, mode, S, W, t, cap, total, ext);
}
int batch_uniform_states(const pj_batch* b, int mode, int S, int W) { return uniform_states(b, mode, S, W); }
int batch_lds_limit(const pj_batch* b) { return lds_max_of(b); }

}  // namespace pj

extern "C" {

pj_status pj_batch_create(pj_batch** out) {
    if (!out) return fail(PJ_E_INVALID, "NULL output handle");
    *out = new (std::nothrow) pj_batch();
    if (!*out) return fail(PJ_E_NOMEM, "out of host memory");
    g_err.clear();
    return PJ_OK;
}

void pj_batch_free(pj_batch* b) {
    if (!b) return;
    b->drop_graph();
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->d_segs) (void)hipFree(b->d_segs);
    delete b;
}

pj_status pj_batch_add(pj_batch* b, const pj_mech* mech, int64_t n_states, const double* d_state,
                       const double* d_param, double* d_out, double* d_dstate_or_null,
                       const double* d_v_or_null, double* d_grad_or_null) {
    if (!b || !mech) return fail(PJ_E_INVALID, "NULL batch or mechanism");
    if (n_states < 0) return fail(PJ_E_INVALID, "negative n_states");
    if (!b->segs.empty() && mech->m.device != b->segs[0].mech->m.device)
        return fail(PJ_E_INVALID, "all mechanisms of a batch must live on one device");
    b->segs.push_back({mech, n_states, d_state, d_param, d_out, d_dstate_or_null, d_v_or_null, d_grad_or_null});
    b->table_valid = false;
    b->drop_graph();
    g_err.clear();
    return PJ_OK;
}

pj_status pj_batch_clear(pj_batch* b) {
    if (!b) return fail(PJ_E_INVALID, "NULL batch");
    b->segs.clear();
    b->table_valid = false;
    b->drop_graph();
    g_err.clear();
    return PJ_OK;
}

int pj_batch_size(const pj_batch* b) { return b ? (int)b->segs.size() : -1; }

pj_status pj_batch_set_launch(pj_batch* b, int mode, int states_per_group, int waves_per_group) {
    if (!b) return fail(PJ_E_INVALID, "NULL batch");
    if (!batch_mode(mode)) return fail(PJ_E_INVALID, "bad mode");
    if (states_per_group != 0 && (states_per_group < 1 || states_per_group > pj::BATCH_MAX_S ||
                                  (states_per_group & (states_per_group - 1))))
        return fail(PJ_E_INVALID, "states_per_group must be 0 or a power of two up to 16");
    if (waves_per_group < 0 || waves_per_group > 8)
        return fail(PJ_E_INVALID, "waves_per_group must be 0 (automatic) or 1 to 8");
    b->user_S[mode] = states_per_group;
    b->user_W[mode] = waves_per_group;
    b->drop_graph();
    g_err.clear();
    return PJ_OK;
}

int pj_batch_launch_shape(const pj_batch* b, int mode, int* states_per_group, int* waves_per_group) {
    if (!b || !batch_mode(mode) || b->segs.empty()) return -1;
    int S, W;
    batch_shape(b, mode, S, W);
    if (states_per_group) *states_per_group = S;
    if (waves_per_group) *waves_per_group = W;
    return 0;
}

int pj_batch_segment_states(const pj_batch* b, int mode, int segment) {
    if (!b || !batch_mode(mode) || segment < 0 || segment >= (int)b->segs.size()) return -1;
    int S, W;
    batch_shape(b, mode, S, W);
    return make_plan(b, mode, S, W).states(b->segs[(size_t)segment]);
}

pj_status pj_batch_set_strategy(pj_batch* b, int mode, int per_segment) {
    if (!b) return fail(PJ_E_INVALID, "NULL batch");
    if (!batch_mode(mode)) return fail(PJ_E_INVALID, "bad mode");
    if (per_segment != 0 && per_segment != 1) return fail(PJ_E_INVALID, "per_segment must be 0 or 1");
    b->per_seg[mode] = per_segment;
    b->drop_graph();
    g_err.clear();
    return PJ_OK;
}

int pj_batch_strategy(const pj_batch* b, int mode) {
    if (!b || !batch_mode(mode)) return -1;
    return b->per_seg[mode];
}

pj_status pj_batch_eval(pj_batch* b, int mode, pj_form form, pj_layout layout, pj_stream stream) {
    if (!b) return fail(PJ_E_INVALID, "NULL batch");
    pj_status r = check_segments(b, mode, form, layout);
    if (r != PJ_OK) return r;
    if (b->segs.empty()) { g_err.clear(); return PJ_OK; }
    int S, W;
    batch_shape(b, mode, S, W);
    if (!b->per_seg[mode] && batch_lds(b, mode, S, W) > lds_max_of(b))
        return fail(PJ_E_UNSUPPORTED, "a segment's working set exceeds the LDS of one workgroup");
    r = enqueue_mode(b, mode, form, layout, S, W, (hipStream_t)stream);
    if (r == PJ_OK) g_err.clear();
    return r;
}

pj_status pj_batch_eval_graph(pj_batch* b, int mode, pj_form form, pj_layout layout, pj_stream stream) {
    if (!b) return fail(PJ_E_INVALID, "NULL batch");
    pj_status r = check_segments(b, mode, form, layout);
    if (r != PJ_OK) return r;
    if (b->segs.empty()) { g_err.clear(); return PJ_OK; }
    int S, W;
    batch_shape(b, mode, S, W);
    const int ps = b->per_seg[mode];
    if (!ps && batch_lds(b, mode, S, W) > lds_max_of(b))
        return fail(PJ_E_UNSUPPORTED, "a segment's working set exceeds the LDS of one workgroup");
    if (!b->exec || b->g_mode != mode || b->g_form != form || b->g_layout != layout || b->g_S != S || b->g_W != W ||
        b->g_per_seg != ps) {
        b->drop_graph();
        if (!ps) {
            r = upload_table(b, mode, S, W);   // synchronous, outside the capture
            if (r != PJ_OK) return r;
        }
        if (!b->capture_stream && hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(PJ_E_DEVICE, "hipStreamCreate failed");
        hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        r = enqueue_mode(b, mode, form, layout, S, W, b->capture_stream);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(b->capture_stream, &gr);
        if (r != PJ_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return r;
        }
        if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        b->graph = gr;
        e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->drop_graph();
            return fail(PJ_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        b->g_mode = mode;
        b->g_form = form;
        b->g_layout = layout;
        b->g_S = S;
        b->g_W = W;
        b->g_per_seg = ps;
    }
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    g_err.clear();
    return PJ_OK;
}

pj_status pj_batch_autotune(pj_batch* b, int mode, pj_form form, pj_layout layout, int reps, pj_stream stream,
                            int* states_per_group, int* waves_per_group, float* ms) {
    if (!b) return fail(PJ_E_INVALID, "NULL batch");
    if (reps < 1) return fail(PJ_E_INVALID, "reps must be at least 1");
    pj_status r = check_segments(b, mode, form, layout);
    if (r != PJ_OK) return r;
    if (b->segs.empty()) return fail(PJ_E_INVALID, "empty batch");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(PJ_E_DEVICE, "hipEventCreate failed");
    }
    const int mx = lds_max_of(b);
    int bS = 0, bW = 0, pS = 0, pW = 0;
    float best = -1.0f, bestp = -1.0f;
    pj_status err = PJ_OK;
    // every persistent launch shape that fits (S > 0), then one launch per
    // segment at each mechanism's current shape (S = 0 below); the best
    // persistent shape is kept for the mode either way
    for (int S = 1; S <= 2 * batch_cap(mode) && err == PJ_OK; S *= 2)
        for (int W = 1; W <= 8 && err == PJ_OK; ++W) {
            const bool segs_each = S == 2 * batch_cap(mode);
            if (segs_each && W > 1) break;
            if (!segs_each && batch_lds(b, mode, S, W) > mx) continue;
            auto run = [&]() {
                return segs_each ? enqueue_segments(b, mode, form, layout, st) : enqueue(b, mode, form, layout, S, W, st);
            };
            err = run();   // warm-up
            hipError_t e = err == PJ_OK ? hipEventRecord(e0, st) : hipSuccess;
            for (int k = 0; k < reps && err == PJ_OK && e == hipSuccess; ++k) err = run();
            if (err != PJ_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) { err = fail(PJ_E_DEVICE, std::string("autotuning: ") + hipGetErrorString(e)); break; }
            t /= (float)reps;
            if (!segs_each && (bestp < 0.0f || t < bestp)) {
                bestp = t;
                pS = S;
                pW = W;
            }
            if (best < 0.0f || t < best) {
                best = t;
                bS = segs_each ? 0 : S;
                bW = segs_each ? 0 : W;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != PJ_OK) return err;
    b->per_seg[mode] = bS == 0 ? 1 : 0;
    if (pS) {
        b->user_S[mode] = pS;
        b->user_W[mode] = pW;
    }
    b->drop_graph();
    if (states_per_group) *states_per_group = bS;
    if (waves_per_group) *waves_per_group = bW;
    if (ms) *ms = best;
    g_err.clear();
    return PJ_OK;
}

const char* pj_batch_last_error(void) { return g_err.c_str(); }

}  // extern "C"
