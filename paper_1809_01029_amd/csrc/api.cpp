// C-ABI entry points (declared in include/pjac.h): argument checking, launch
// shape, and dispatch to the kernels.  No call here synchronises the host
// except pj_mech_load, which uploads the tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "internal.h"

namespace {

thread_local std::string g_err;

pj_status fail(pj_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

bool pow2_upto(int v, int mx) { return v >= 1 && v <= mx && (v & (v - 1)) == 0; }

constexpr int MAX_S = 64, MAX_WAVES = 8;

// The kernel that evaluates `mode` for a mechanism: the run-time slot search
// and the fixed-order additions have kernels of their own, and so has a call
// with its own Arrhenius parameters.
int kernel_mode(const pj::Mechanism& m, int mode, bool per_call_arrhenius) {
    if (per_call_arrhenius) return mode == pj::MODE_SRC ? pj::MODE_SRC_P : pj::MODE_ADJ_P;
    if (mode == pj::MODE_DENSE && m.dense_unroll == 16 && m.S[mode] <= 4) return pj::MODE_DENSE_U16;
    if (mode == pj::MODE_SPARSE && m.dm.lsearch) return pj::MODE_SPARSE_LS;
    if (m.dm.det && mode == pj::MODE_SRC) return pj::MODE_SRC_DET;
    if (m.dm.det && mode == pj::MODE_SPARSE) return pj::MODE_SPARSE_DET;
    return mode;
}

// the most states per workgroup a kernel mode is built for
int max_states(int kmode) {
    if (kmode == pj::MODE_SPARSE_LS || kmode == pj::MODE_SRC_DET || kmode == pj::MODE_SPARSE_DET) return 4;
    if (pj::base_mode(kmode) == pj::MODE_ADJ) return pj::MAX_S_ADJ;
    return MAX_S;
}

}  // namespace

namespace pj {

// Waves per workgroup for S states per workgroup: enough that a compute unit
// holds about 8 resident waves given how many workgroups fit in its LDS, and
// at least S/64 so that every state has a lane.
static int default_waves(const Mechanism& m, int mode, int S, bool gr) {
    int w = S > 64 ? S / 64 : 1;
    while (w < MAX_WAVES) {
        const int64_t l = lds_bytes(m.dm, mode, S, w, gr);
        if (l > m.lds_max || (m.lds_max / l) * w >= 8) break;
        w *= 2;
    }
    return w;
}

// Launch shape of each mode.  States per workgroup S: the most (4, 2 or 1)
// whose interleaved working set fits the LDS of one workgroup; waves per
// workgroup as default_waves.  A user setting overrides either choice when it
// fits.  The adjoint keeps its per-reaction parameter sums in LDS when they
// fit beside one state's working set.
void choose_launch(Mechanism& m) {
    m.adj_grad_in_lds = lds_bytes(m.dm, MODE_ADJ, 1, 1, true) <= m.lds_max;
    for (int mode = 0; mode < N_MODES; ++mode) {
        const bool gr = mode == MODE_ADJ && m.adj_grad_in_lds;
        auto L = [&](int S, int w) { return lds_bytes(m.dm, mode, S, w, gr); };
        int S = 1;
        for (int c = 4; c >= 1; c >>= 1)
            if (L(c, 1) <= m.lds_max) { S = c; break; }
        const int maxS = max_states(kernel_mode(m, mode, false));
        if (m.user_S && m.user_S <= maxS && L(m.user_S, m.user_waves ? m.user_waves : 1) <= m.lds_max)
            S = m.user_S;
        int w = m.user_waves ? m.user_waves : default_waves(m, mode, S, gr);
        if (L(S, w) > m.lds_max) w = default_waves(m, mode, S, gr);
        m.S[mode] = S;
        m.waves[mode] = w;
        m.lds[mode] = L(S, w);
    }
}

}  // namespace pj

namespace {

pj_status eval(const pj_mech* mech, int mode, pj_form form, pj_layout layout, int64_t n,
               const double* state, const double* param, double* dstate, double* jac,
               pj_stream stream, const double* vin = nullptr, double* grad = nullptr,
               const double* arr = nullptr) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (form != PJ_CONP && form != PJ_CONV) return fail(PJ_E_INVALID, "bad form");
    if (layout != PJ_LAYOUT_F && layout != PJ_LAYOUT_C) return fail(PJ_E_INVALID, "bad layout");
    if (n < 0) return fail(PJ_E_INVALID, "negative n_states");
    if (n == 0) { g_err.clear(); return PJ_OK; }
    if (!state || !param) return fail(PJ_E_INVALID, "NULL state or parameter");
    if (mode == pj::MODE_SRC && !dstate) return fail(PJ_E_INVALID, "NULL output");
    if (mode != pj::MODE_SRC && !jac)
        return fail(PJ_E_INVALID, mode == pj::MODE_ADJ ? "NULL J^T v output" : "NULL Jacobian output");
    if (mode == pj::MODE_ADJ && !vin) return fail(PJ_E_INVALID, "NULL vector v");
    const pj::Mechanism& m = mech->m;
    if (!m.dbuf) return fail(PJ_E_INVALID, "mechanism not uploaded to a device");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m.device)
        return fail(PJ_E_INVALID, "the current HIP device is not the one the mechanism was loaded on");
    const int64_t lds = m.lds[mode];
    if (lds > m.lds_max)
        return fail(PJ_E_UNSUPPORTED, "per-state working set (" + std::to_string(lds) +
                                          " B) exceeds the LDS of one workgroup");
    // the hot loop of the static map carries no trace of the run-time search,
    // the fixed-order additions or per-call parameters: kernels of their own
    const int kmode = kernel_mode(m, mode, arr != nullptr);
    const int S = std::min(m.S[mode], max_states(kmode));
    // a call with its own Arrhenius parameters runs on a copy of the device
    // description that points at them (the mechanism itself is not touched)
    pj::DevMech dm = m.dm;
    dm.arr = pj::gptr(arr);
    hipError_t e = pj::launch(dm, kmode, form, layout, S, n, state, param, dstate, jac, vin, grad,
                              m.adj_grad_in_lds ? 1 : 0, m.waves[mode], pj::lds_bytes(m.dm, mode, S, m.waves[mode],
                              m.adj_grad_in_lds), (hipStream_t)stream);
    if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    g_err.clear();
    return PJ_OK;
}

}  // namespace

extern "C" {

pj_status pj_mech_parse_ex(const char* desc_path, int options, pj_mech** out) {
    if (!out) return fail(PJ_E_INVALID, "NULL output handle");
    *out = nullptr;
    if (!desc_path) return fail(PJ_E_INVALID, "NULL path");
    if (options & ~(PJ_OPT_APPROX_JACOBIAN | PJ_OPT_CCS | PJ_OPT_LINEAR_SEARCH | PJ_OPT_DETERMINISTIC))
        return fail(PJ_E_INVALID, "unknown option bits");
    pj_mech* h = new (std::nothrow) pj_mech();
    if (!h) return fail(PJ_E_NOMEM, "out of host memory");
    h->m.opts = options;
    std::string err;
    pj_status st = pj::build_mechanism(desc_path, h->m, err);
    if (st != PJ_OK) {
        pj_mech_free(h);
        return fail(st, err);
    }
    *out = h;
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_upload(pj_mech* mech) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (mech->m.dbuf) return fail(PJ_E_INVALID, "mechanism already uploaded");
    std::string err;
    pj_status st = pj::upload_mechanism(mech->m, err);
    if (st != PJ_OK) {
        if (mech->m.dbuf) { (void)hipFree(mech->m.dbuf); mech->m.dbuf = nullptr; }
        return fail(st, err);
    }
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_parse(const char* desc_path, pj_mech** out) { return pj_mech_parse_ex(desc_path, 0, out); }

int pj_mech_options(const pj_mech* mech) { return mech ? mech->m.opts : -1; }

pj_status pj_mech_load(const char* desc_path, pj_mech** out) { return pj_mech_load_ex(desc_path, 0, out); }

pj_status pj_mech_load_ex(const char* desc_path, int options, pj_mech** out) {
    pj_status st = pj_mech_parse_ex(desc_path, options, out);
    if (st != PJ_OK) return st;
    st = pj_mech_upload(*out);
    if (st != PJ_OK) {
        std::string keep = g_err;
        pj_mech_free(*out);
        *out = nullptr;
        return fail(st, keep);
    }
    return PJ_OK;
}

void pj_mech_free(pj_mech* mech) {
    if (!mech) return;
    if (mech->m.dbuf) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != mech->m.device) (void)hipSetDevice(mech->m.device);
        (void)hipFree(mech->m.dbuf);
        if (cur >= 0 && cur != mech->m.device) (void)hipSetDevice(cur);
    }
    delete mech;
}

int pj_mech_n_species(const pj_mech* mech) { return mech ? mech->m.ns : -1; }
int pj_mech_n_reactions(const pj_mech* mech) { return mech ? mech->m.nr : -1; }
int pj_mech_state_size(const pj_mech* mech) { return mech ? mech->m.ns + 1 : -1; }

pj_status pj_mech_jac_pattern(const pj_mech* mech, int64_t* nnz, const int32_t** row_ptr,
                              const int32_t** col_idx) {
    if (!mech || !nnz || !row_ptr || !col_idx) return fail(PJ_E_INVALID, "NULL argument");
    *nnz = mech->m.nnz;
    *row_ptr = mech->m.row_ptr.data();
    *col_idx = mech->m.col_idx.data();
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_jac_pattern_ccs(const pj_mech* mech, int64_t* nnz, const int32_t** col_ptr,
                                  const int32_t** row_idx) {
    if (!mech || !nnz || !col_ptr || !row_idx) return fail(PJ_E_INVALID, "NULL argument");
    *nnz = mech->m.nnz;
    *col_ptr = mech->m.col_ptr.data();
    *row_idx = mech->m.row_idx.data();
    g_err.clear();
    return PJ_OK;
}

pj_status pj_eval_source(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                         const double* d_state, const double* d_param, double* d_dstate,
                         pj_stream stream) {
    return eval(mech, pj::MODE_SRC, form, layout, n_states, d_state, d_param, d_dstate, nullptr,
                stream);
}

pj_status pj_eval_jacobian_sparse(const pj_mech* mech, pj_form form, pj_layout layout,
                                  int64_t n_states, const double* d_state, const double* d_param,
                                  double* d_jac_vals, double* d_dstate_or_null, pj_stream stream) {
    return eval(mech, pj::MODE_SPARSE, form, layout, n_states, d_state, d_param, d_dstate_or_null,
                d_jac_vals, stream);
}

pj_status pj_eval_jacobian_dense(const pj_mech* mech, pj_form form, pj_layout layout,
                                 int64_t n_states, const double* d_state, const double* d_param,
                                 double* d_jac, double* d_dstate_or_null, pj_stream stream) {
    return eval(mech, pj::MODE_DENSE, form, layout, n_states, d_state, d_param, d_dstate_or_null,
                d_jac, stream);
}

pj_status pj_eval_adjoint(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                          const double* d_state, const double* d_param, const double* d_v,
                          double* d_jtv, double* d_grad_or_null, double* d_dstate_or_null,
                          pj_stream stream) {
    if (n_states == 0 && mech && d_grad_or_null && mech->m.dbuf) {
        // an empty batch still defines the gradient sums: zero
        hipError_t e = pj::zero_async(d_grad_or_null, 3 * (int64_t)mech->m.nr, (hipStream_t)stream);
        if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("zeroing the gradient failed: ") + hipGetErrorString(e));
    }
    return eval(mech, pj::MODE_ADJ, form, layout, n_states, d_state, d_param, d_dstate_or_null, d_jtv,
                stream, d_v, d_grad_or_null);
}

pj_status pj_eval_source_arrhenius(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                                   const double* d_state, const double* d_param, const double* d_arrhenius,
                                   double* d_dstate, pj_stream stream) {
    if (!d_arrhenius) return fail(PJ_E_INVALID, "NULL Arrhenius parameters");
    return eval(mech, pj::MODE_SRC, form, layout, n_states, d_state, d_param, d_dstate, nullptr, stream,
                nullptr, nullptr, d_arrhenius);
}

pj_status pj_eval_adjoint_arrhenius(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                                    const double* d_state, const double* d_param, const double* d_arrhenius,
                                    const double* d_v, double* d_jtv, double* d_grad_or_null,
                                    double* d_dstate_or_null, pj_stream stream) {
    if (!d_arrhenius) return fail(PJ_E_INVALID, "NULL Arrhenius parameters");
    if (n_states == 0 && mech && d_grad_or_null && mech->m.dbuf) {
        hipError_t e = pj::zero_async(d_grad_or_null, 3 * (int64_t)mech->m.nr, (hipStream_t)stream);
        if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("zeroing the gradient failed: ") + hipGetErrorString(e));
    }
    return eval(mech, pj::MODE_ADJ, form, layout, n_states, d_state, d_param, d_dstate_or_null, d_jtv,
                stream, d_v, d_grad_or_null, d_arrhenius);
}

pj_status pj_mech_set_arrhenius(pj_mech* mech, const double* lnA, const double* b, const double* theta) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    pj::Mechanism& m = mech->m;
    for (int i = 0; i < m.nr; ++i) {
        if (lnA) m.rx[i].lnA = lnA[i];
        if (b) m.rx[i].b = b[i];
        if (theta) m.rx[i].theta = theta[i];
    }
    if (m.dbuf) {
        for (int p = 0; p < m.nr; ++p) {
            const auto& r = m.rx[m.order[p]];
            m.h_rec[p].lnA = r.lnA;
            m.h_rec[p].b = r.b;
            m.h_rec[p].theta = r.theta;
        }
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != m.device && hipSetDevice(m.device) != hipSuccess)
            return fail(PJ_E_DEVICE, "cannot select the mechanism's device");
        hipError_t e = hipMemcpy((unsigned char*)m.dbuf + m.off_rec, m.h_rec.data(),
                                 m.h_rec.size() * sizeof(pj::RxnRec), hipMemcpyHostToDevice);
        if (cur >= 0 && cur != m.device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("update of the reaction table failed: ") + hipGetErrorString(e));
    }
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_get_arrhenius(const pj_mech* mech, double* lnA, double* b, double* theta) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    for (int i = 0; i < mech->m.nr; ++i) {
        if (lnA) lnA[i] = mech->m.rx[i].lnA;
        if (b) b[i] = mech->m.rx[i].b;
        if (theta) theta[i] = mech->m.rx[i].theta;
    }
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_set_launch(pj_mech* mech, int states_per_group, int waves_per_group) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (states_per_group && !pow2_upto(states_per_group, MAX_S))
        return fail(PJ_E_INVALID, "states_per_group must be 0 or a power of two up to 64");
    if (waves_per_group < 0 || waves_per_group > MAX_WAVES)
        return fail(PJ_E_INVALID, "waves_per_group must be 0 (automatic) or 1 to 8");
    mech->m.user_S = states_per_group;
    mech->m.user_waves = waves_per_group;
    if (mech->m.dbuf) {
        pj::choose_launch(mech->m);
    } else {
        // provisional until the upload measures the LDS the modes need
        for (int mode = 0; mode < pj::N_MODES; ++mode) {
            mech->m.S[mode] = states_per_group ? states_per_group : 1;
            if (mode == pj::MODE_ADJ && mech->m.S[mode] > pj::MAX_S_ADJ) mech->m.S[mode] = pj::MAX_S_ADJ;
            mech->m.waves[mode] = waves_per_group ? waves_per_group : 1;
        }
    }
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_set_waves_per_state(pj_mech* mech, int waves_per_state) {
    if (waves_per_state != 0 && !pow2_upto(waves_per_state, 4))
        return fail(PJ_E_INVALID, "waves_per_state must be 0, 1, 2 or 4");
    return pj_mech_set_launch(mech, waves_per_state ? 1 : 0, waves_per_state);
}

int pj_mech_waves_per_state(const pj_mech* mech, int for_jacobian) {
    if (!mech) return -1;
    const int mode = for_jacobian ? pj::MODE_SPARSE : pj::MODE_SRC;
    return mech->m.S[mode] == 1 ? mech->m.waves[mode] : -1;
}

pj_status pj_mech_set_dense_unroll(pj_mech* mech, int entries) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (entries != 0 && entries != 8 && entries != 16)
        return fail(PJ_E_INVALID, "entries must be 0 (default, 16), 8 or 16");
    mech->m.dense_unroll = entries == 8 ? 8 : 16;
    g_err.clear();
    return PJ_OK;
}

int pj_mech_dense_unroll(const pj_mech* mech) { return mech ? mech->m.dense_unroll : -1; }

int pj_mech_launch_shape(const pj_mech* mech, int mode, int* states_per_group, int* waves_per_group) {
    if (!mech || mode < 0 || mode >= pj::N_MODES) return -1;
    if (states_per_group) *states_per_group = mech->m.S[mode];
    if (waves_per_group) *waves_per_group = mech->m.waves[mode];
    return 0;
}

}  // extern "C"

namespace {

// time every launch shape that fits for `mode` and keep the fastest
pj_status autotune(pj_mech* mech, int mode, pj_form form, pj_layout layout, int64_t n_states,
                   const double* d_state, const double* d_param, double* dst, double* jac, const double* vin,
                   double* grad, int reps, pj_stream stream, int* states_per_group, int* waves_per_group,
                   float* ms) {
    if (reps < 1) return fail(PJ_E_INVALID, "reps must be at least 1");
    if (n_states < 1) return fail(PJ_E_INVALID, "autotuning needs at least one state");
    pj::Mechanism& m = mech->m;
    // validate the arguments once with the current shape
    pj_status st = eval(mech, mode, form, layout, n_states, d_state, d_param, dst, jac, stream, vin, grad);
    if (st != PJ_OK) return st;
    const bool gr = mode == pj::MODE_ADJ && m.adj_grad_in_lds;
    const int kmode0 = kernel_mode(m, mode, false);
    const int maxS = max_states(kmode0);
    // the dense output's unroll width is a dimension of the search (8, 16)
    const int n_du = mode == pj::MODE_DENSE ? 2 : 1;
    int best_du = m.dense_unroll;
    hipStream_t hs = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(PJ_E_DEVICE, "hipEventCreate failed");
    }
    int best_S = m.S[mode], best_w = m.waves[mode];
    float best = -1.0f;
    std::string err;
    for (int S = 1; S <= maxS && err.empty(); S *= 2) {
        for (int w = 1; w <= MAX_WAVES * n_du && err.empty(); ++w) {
            const int du = w > MAX_WAVES ? 8 : 16;
            const int wv = w > MAX_WAVES ? w - MAX_WAVES : w;
            const int kmode = n_du == 2 ? (du == 16 ? pj::MODE_DENSE_U16 : pj::MODE_DENSE) : kmode0;
            if (kmode == pj::MODE_DENSE_U16 && S > 4) continue;   // built for at most 4 states
            const int64_t l = pj::lds_bytes(m.dm, mode, S, wv, gr);
            if (l > m.lds_max) continue;
            auto go = [&]() {
                return pj::launch(m.dm, kmode, form, layout, S, n_states, d_state, d_param, dst, jac, vin, grad,
                                  gr ? 1 : 0, wv, l, hs);
            };
            hipError_t e = go();
            if (e == hipSuccess) e = hipEventRecord(e0, hs);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = go();
            if (e == hipSuccess) e = hipEventRecord(e1, hs);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) {
                err = std::string("autotuning launch failed: ") + hipGetErrorString(e);
                break;
            }
            t /= (float)reps;
            if (best < 0.0f || t < best) {
                best = t;
                best_S = S;
                best_w = wv;
                best_du = du;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!err.empty()) return fail(PJ_E_DEVICE, err);
    m.S[mode] = best_S;
    m.waves[mode] = best_w;
    m.lds[mode] = pj::lds_bytes(m.dm, mode, best_S, best_w, gr);
    if (mode == pj::MODE_DENSE) m.dense_unroll = best_du;
    if (states_per_group) *states_per_group = best_S;
    if (waves_per_group) *waves_per_group = best_w;
    if (ms) *ms = best;
    g_err.clear();
    return PJ_OK;
}

}  // namespace

extern "C" {

pj_status pj_mech_autotune(pj_mech* mech, int mode, pj_form form, pj_layout layout, int64_t n_states,
                           const double* d_state, const double* d_param, double* d_out,
                           double* d_dstate_or_null, int reps, pj_stream stream,
                           int* states_per_group, int* waves_per_group, float* ms) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (mode < pj::MODE_SRC || mode > pj::MODE_DENSE) return fail(PJ_E_INVALID, "bad mode");
    double* dst = mode == pj::MODE_SRC ? d_out : d_dstate_or_null;
    double* jac = mode == pj::MODE_SRC ? nullptr : d_out;
    return autotune(mech, mode, form, layout, n_states, d_state, d_param, dst, jac, nullptr, nullptr, reps, stream,
                    states_per_group, waves_per_group, ms);
}

pj_status pj_mech_autotune_adjoint(pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                                   const double* d_state, const double* d_param, const double* d_v,
                                   double* d_jtv, double* d_grad_or_null, int reps, pj_stream stream,
                                   int* states_per_group, int* waves_per_group, float* ms) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    return autotune(mech, pj::MODE_ADJ, form, layout, n_states, d_state, d_param, nullptr, d_jtv, d_v,
                    d_grad_or_null, reps, stream, states_per_group, waves_per_group, ms);
}

int64_t pj_mech_lds_bytes(const pj_mech* mech, int for_jacobian) {
    if (!mech) return -1;
    return for_jacobian ? mech->m.lds[pj::MODE_SPARSE] : mech->m.lds[pj::MODE_SRC];
}

const char* pj_last_error(void) { return g_err.c_str(); }

}  // extern "C"
