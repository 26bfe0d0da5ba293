// C-ABI entry points (declared in include/pjac.h): argument checking, launch
// shape, and dispatch to the kernels.  No call here synchronises the host
// except pj_mech_load, which uploads the tables.
#include <hip/hip_runtime.h>

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

bool valid_wps(int w) { return w == 1 || w == 2 || w == 4; }

// Automatic launch shape: the fewest waves per state that still give a
// compute unit at least 8 resident waves (two per SIMD) given how many
// states fit in its LDS at once.
int auto_wps(int64_t lds_bytes, int lds_max) {
    const int64_t blocks = lds_bytes > 0 ? lds_max / lds_bytes : 32;
    for (int w = 1; w <= 4; w *= 2)
        if (blocks * w >= 8) return w;
    return 4;
}

pj_status eval(const pj_mech* mech, int mode, pj_form form, pj_layout layout, int64_t n,
               const double* state, const double* param, double* dstate, double* jac,
               pj_stream stream) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (form != PJ_CONP && form != PJ_CONV) return fail(PJ_E_INVALID, "bad form");
    if (layout != PJ_LAYOUT_F && layout != PJ_LAYOUT_C) return fail(PJ_E_INVALID, "bad layout");
    if (n < 0) return fail(PJ_E_INVALID, "negative n_states");
    if (n == 0) { g_err.clear(); return PJ_OK; }
    if (!state || !param) return fail(PJ_E_INVALID, "NULL state or parameter");
    if (mode == pj::MODE_SRC && !dstate) return fail(PJ_E_INVALID, "NULL output");
    if (mode != pj::MODE_SRC && !jac) return fail(PJ_E_INVALID, "NULL Jacobian output");
    const pj::Mechanism& m = mech->m;
    if (!m.dbuf) return fail(PJ_E_INVALID, "mechanism not uploaded to a device");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m.device)
        return fail(PJ_E_INVALID, "the current HIP device is not the one the mechanism was loaded on");
    int64_t lds = mode == pj::MODE_SRC ? m.lds_src : mode == pj::MODE_SPARSE ? m.lds_jac : m.lds_dense;
    if (lds > m.lds_max)
        return fail(PJ_E_UNSUPPORTED, "per-state working set (" + std::to_string(lds) +
                                          " B) exceeds the LDS of one workgroup");
    int wps = mode == pj::MODE_SRC ? m.wps_src : m.wps_jac;
    hipError_t e = pj::launch(m.dm, mode, form, layout, n, state, param, dstate, jac, wps, lds,
                              (hipStream_t)stream);
    if (e != hipSuccess) return fail(PJ_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    g_err.clear();
    return PJ_OK;
}

}  // namespace

extern "C" {

pj_status pj_mech_parse(const char* desc_path, pj_mech** out) {
    if (!out) return fail(PJ_E_INVALID, "NULL output handle");
    *out = nullptr;
    if (!desc_path) return fail(PJ_E_INVALID, "NULL path");
    pj_mech* h = new (std::nothrow) pj_mech();
    if (!h) return fail(PJ_E_NOMEM, "out of host memory");
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
    if (!mech->m.wps_user) {
        mech->m.wps_src = auto_wps(mech->m.lds_src, mech->m.lds_max);
        mech->m.wps_jac = auto_wps(mech->m.lds_jac, mech->m.lds_max);
    }
    g_err.clear();
    return PJ_OK;
}

pj_status pj_mech_load(const char* desc_path, pj_mech** out) {
    pj_status st = pj_mech_parse(desc_path, out);
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

pj_status pj_mech_set_waves_per_state(pj_mech* mech, int waves_per_state) {
    if (!mech) return fail(PJ_E_INVALID, "NULL mechanism");
    if (waves_per_state == 0) {
        if (mech->m.dbuf) {
            mech->m.wps_src = auto_wps(mech->m.lds_src, mech->m.lds_max);
            mech->m.wps_jac = auto_wps(mech->m.lds_jac, mech->m.lds_max);
        }
        mech->m.wps_user = false;
    } else {
        if (!valid_wps(waves_per_state)) return fail(PJ_E_INVALID, "waves_per_state must be 1, 2 or 4");
        mech->m.wps_src = mech->m.wps_jac = waves_per_state;
        mech->m.wps_user = true;
    }
    g_err.clear();
    return PJ_OK;
}

int pj_mech_waves_per_state(const pj_mech* mech, int for_jacobian) {
    if (!mech) return -1;
    return for_jacobian ? mech->m.wps_jac : mech->m.wps_src;
}

int64_t pj_mech_lds_bytes(const pj_mech* mech, int for_jacobian) {
    if (!mech) return -1;
    return for_jacobian ? mech->m.lds_jac : mech->m.lds_src;
}

const char* pj_last_error(void) { return g_err.c_str(); }

}  // extern "C"
