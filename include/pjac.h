/*
 * pjac.h - C-ABI of the MI355X (gfx950) library that evaluates thermochemical
 * source terms and the analytical sparse / dense chemical-kinetic Jacobian for
 * very many independent thermochemical states, after Curtis, Niemeyer & Sung,
 * "Using SIMD and SIMT vectorization to evaluate sparse chemical kinetic
 * Jacobian matrices and thermochemical source terms" (pyJac v2,
 * arXiv:1809.01029).
 *
 * Problem statement (paper Sec. 2.2).  For a mechanism with Ns species (the
 * last one the bath gas) the state vector has N = Ns + 1 entries:
 *     constant pressure (CONP): Phi = (T, V, n_1 .. n_{Ns-1}),  parameter P
 *     constant volume   (CONV): Phi = (T, P, n_1 .. n_{Ns-1}),  parameter V
 * with T in K, V in m^3, P in Pa and n_k in kmol.  The bath gas moles follow
 * from the ideal-gas law, n_Ns = P V / (R T) - sum_{k<Ns} n_k, where the sum
 * is the exactly rounded sum of the n_k.  The source terms are
 *     dT/dt  = -sum_k e_k wdot_k / sum_k [C]_k chat_k     (e = H or U, chat = Cp or Cv)
 *     dn_k/dt = V wdot_k,   wdot_k = sum_i nu_ki c_i R_i   (Sec. 2.2)
 *     CONP: dV/dt = V/T dT/dt + V R T / P * Omega
 *     CONV: dP/dt = P/T dT/dt + R T * Omega,   Omega = sum_{k<Ns} (1 - W_k/W_Ns) wdot_k
 * and the Jacobian is J[i][j] = d(dPhi_i/dt)/dPhi_j (Sec. 2.2), stored either
 * on a fixed per-mechanism CSR pattern (Sec. 3.4) or dense.
 * Units: SI with kmol, R = 8314.462618 J/(kmol K), reference pressure 101325 Pa.
 *
 * Layouts (Sec. 2.1, data ordering):
 *   PJ_LAYOUT_C  state-major: state[s*N + i], dstate[s*N + i],
 *                CSR values jac[s*nnz + e], dense jac[s*N*N + i*N + j]
 *   PJ_LAYOUT_F  variable-major (each variable of all states contiguous):
 *                state[i*n + s], dstate[i*n + s], CSR values jac[e*n + s],
 *                dense jac[s + n*(i + N*j)]  (Fortran order of (state, row, col))
 * param[s] is one value per state in both layouts.
 *
 * Conventions.
 *   - Every d_* pointer is device memory owned by the caller; the library never
 *     frees it.  The mechanism handle and the pattern arrays it hands out are
 *     owned by the library until pj_mech_free.
 *   - Evaluation calls are asynchronous on the given HIP stream and never
 *     synchronise the host.  n_states == 0 is a no-op returning PJ_OK.
 *   - Errors are status codes; pj_last_error() gives a thread-local message.
 *     NULL pointers (with n_states > 0), n_states < 0, bad enums, a NULL
 *     handle, a handle that was not uploaded, or a current HIP device other
 *     than the one the mechanism was uploaded to give PJ_E_INVALID; a failed
 *     launch gives PJ_E_DEVICE.
 *   - Non-physical inputs (T <= 0, a negative bath gas) are not checked on the
 *     device; NaN and inf propagate to the outputs.
 */
#ifndef PJAC_H
#define PJAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pj_mech pj_mech; /* opaque, library-owned */

/* HIP stream handle (hipStream_t); NULL is the default stream. */
typedef void* pj_stream;

typedef enum { PJ_CONP = 0, PJ_CONV = 1 } pj_form;
typedef enum { PJ_LAYOUT_F = 0, PJ_LAYOUT_C = 1 } pj_layout;

typedef enum {
    PJ_OK = 0,
    PJ_E_INVALID = 1,     /* bad argument */
    PJ_E_PARSE = 2,       /* malformed mechanism description */
    PJ_E_UNBALANCED = 3,  /* a reaction does not conserve elements */
    PJ_E_DEVICE = 4,      /* HIP error (allocation, copy, launch) */
    PJ_E_NOMEM = 5,       /* host allocation failed */
    PJ_E_UNSUPPORTED = 6  /* mechanism outside what the kernels handle */
} pj_status;

/*
 * Load a mechanism description (the text format written by the package's
 * synthetic generator: species with NASA 7-coefficient thermodynamics,
 * reactions of type elementary, third-body, falloff with the Lindemann, Troe
 * or SRI form, chemically activated with the same forms, pressure-dependent
 * Arrhenius (P-Log) and Chebyshev; the reaction types Sec. 2.2 names as
 * supported), check that
 * every reaction conserves elements, derive the device tables and the CSR
 * pattern of the Jacobian (Sec. 3.4), and upload them to the current HIP
 * device.  Synchronous.  On success *out receives a handle; on failure *out is
 * NULL and the status says why.
 * Limits (PJ_E_UNSUPPORTED beyond them): at most 3 distinct species per
 * reaction side, coefficients 1..2, at most 8 third bodies with an efficiency
 * other than one per reaction, at most 64 pressures per P-Log reaction and
 * 16 x 16 Chebyshev coefficients, at most 65534 Jacobian non-zeros, and the
 * per-state working set must fit the device's LDS per workgroup.
 */
pj_status pj_mech_load(const char* desc_path, pj_mech** out);

/*
 * pj_mech_load with options (bitwise or; 0 = pj_mech_load):
 *   PJ_OPT_APPROX_JACOBIAN  the "approximate" Jacobian of Sec. 3.4: the bath
 *       gas's moles are held fixed against the other species' moles (their
 *       dependence on T and V or P kept), so a reaction of the bath gas, or a
 *       bath-gas efficiency other than one, no longer makes rows dense; the
 *       pattern is that form's.
 *   PJ_OPT_CCS  sparse values in column order (the compressed-column storage
 *       the paper pairs with layout F): value k of a state is the entry
 *       (row_idx[k], column c) with col_ptr[c] <= k < col_ptr[c+1], see
 *       pj_mech_jac_pattern_ccs; the CSR arrays still describe the pattern.
 *   PJ_OPT_LINEAR_SEARCH  species-row entries find their CSR slot by
 *       searching the row at run time (the lookup the paper times, Sec. 3.4)
 *       instead of the static slot map: same values, for comparison.
 *   PJ_OPT_DETERMINISTIC  source terms and the sparse Jacobian (and its fused
 *       source terms) bitwise reproducible from run to run at any one launch
 *       shape: the waves of a workgroup add their reactions' contributions to
 *       the shared sums in turn instead of at once (slower; at most 4 states
 *       per workgroup).  Results may still differ in the last bits between
 *       two launch shapes, which split the reactions differently.  Dense,
 *       adjoint, run-time-search, per-call-parameter and pj_batch_eval
 *       evaluations are unaffected (a one-wave workgroup is always
 *       reproducible).
 */
enum { PJ_OPT_APPROX_JACOBIAN = 1, PJ_OPT_CCS = 2, PJ_OPT_LINEAR_SEARCH = 4, PJ_OPT_DETERMINISTIC = 8 };
pj_status pj_mech_load_ex(const char* desc_path, int options, pj_mech** out);
pj_status pj_mech_parse_ex(const char* desc_path, int options, pj_mech** out);
int pj_mech_options(const pj_mech* mech); /* -1 for NULL */

/*
 * The pattern in column order: col_ptr has N+1 entries, row_idx nnz entries
 * with ascending rows in each column; host arrays owned by the mechanism.
 */
pj_status pj_mech_jac_pattern_ccs(const pj_mech* mech, int64_t* nnz, const int32_t** col_ptr,
                                  const int32_t** row_idx);

/*
 * The two halves of pj_mech_load.  pj_mech_parse parses, validates and
 * derives the CSR pattern on the host only (no device needed): the handle can
 * be queried (sizes, pattern) and freed, but not evaluated.  pj_mech_upload
 * derives the device tables and uploads them to the current HIP device
 * (synchronous); PJ_E_INVALID if the mechanism was already uploaded.
 */
pj_status pj_mech_parse(const char* desc_path, pj_mech** out);
pj_status pj_mech_upload(pj_mech* mech);

/* Release a mechanism and its device tables.  NULL is accepted. */
void pj_mech_free(pj_mech* mech);

int pj_mech_n_species(const pj_mech* mech);   /* Ns, or -1 for NULL */
int pj_mech_n_reactions(const pj_mech* mech); /* Nr, or -1 for NULL */
int pj_mech_state_size(const pj_mech* mech);  /* N = Ns + 1, or -1 for NULL */

/*
 * The fixed CSR pattern of the Jacobian (Sec. 3.4): row_ptr has N+1 entries,
 * col_idx has nnz entries with ascending columns in each row.  Rows and
 * columns 0 (T) and 1 (V or P) are dense; species row k holds column j when a
 * reaction with a non-zero net coefficient of k has a rate of progress that
 * depends on [C]_j (j a reactant, a product of a reversible reaction, or a
 * third body whose efficiency differs from the bath gas's); a rate that
 * depends on the bath gas makes the row dense; the diagonal is always held.
 * The arrays are host memory owned by the mechanism.
 */
pj_status pj_mech_jac_pattern(const pj_mech* mech, int64_t* nnz, const int32_t** row_ptr,
                              const int32_t** col_idx);

/*
 * Source terms dPhi/dt (Sec. 2.2) for n_states states.
 * d_state: N*n doubles in `layout`; d_param: n doubles (P for CONP, V for
 * CONV); d_dstate: N*n doubles written in the same layout as d_state.
 */
pj_status pj_eval_source(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                         const double* d_state, const double* d_param, double* d_dstate,
                         pj_stream stream);

/*
 * Analytical Jacobian on the CSR pattern (Sec. 3.4) plus, when
 * d_dstate_or_null is not NULL, the source terms of the same states (one
 * fused pass).  d_jac_vals: nnz*n doubles, [e*n + s] (F) or [s*nnz + e] (C).
 */
pj_status pj_eval_jacobian_sparse(const pj_mech* mech, pj_form form, pj_layout layout,
                                  int64_t n_states, const double* d_state, const double* d_param,
                                  double* d_jac_vals, double* d_dstate_or_null, pj_stream stream);

/*
 * Analytical Jacobian as a dense N x N matrix per state (entries outside the
 * pattern are written as 0), plus optional fused source terms.
 * d_jac: N*N*n doubles, [s + n*(i + N*j)] (F) or [s*N*N + i*N + j] (C).
 */
pj_status pj_eval_jacobian_dense(const pj_mech* mech, pj_form form, pj_layout layout,
                                 int64_t n_states, const double* d_state, const double* d_param,
                                 double* d_jac, double* d_dstate_or_null, pj_stream stream);

/*
 * Adjoint (for calibrating the mechanism against data): for every state the
 * product of the transposed Jacobian with a vector, J^T v, and, summed over
 * the batch, the derivatives of v . dPhi/dt with respect to every reaction's
 * Arrhenius parameters ln A, b and Ea/R (Sec. 2.2's rate constants; for
 * falloff and chemically activated reactions those of the high-pressure
 * limit, the low-pressure limit held fixed; for P-Log and Chebyshev reactions
 * those of the Arrhenius factor that multiplies the tabulated rate).  J^T v
 * is accumulated on chip from each reaction's rate gradient weighted by its
 * stoichiometry and v (the Jacobian itself is never formed), with the same
 * derivatives as pj_eval_jacobian_sparse.
 * d_v: N*n doubles, same layout as d_state; d_jtv: N*n doubles, same layout;
 * d_grad_or_null: NULL, or 3*Nr doubles [ln A (Nr), b (Nr), Ea/R (Nr)] in the
 * description's reaction order, overwritten with the batch sums (workgroups
 * add their partial sums with atomics, so the last bits may vary from run to
 * run); d_dstate_or_null: optional fused source terms.
 */
pj_status pj_eval_adjoint(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                          const double* d_state, const double* d_param, const double* d_v,
                          double* d_jtv, double* d_grad_or_null, double* d_dstate_or_null,
                          pj_stream stream);

/*
 * pj_eval_source and pj_eval_adjoint with the Arrhenius parameters of this
 * call given as a device array instead of the mechanism's tables (what a
 * differentiable calibration needs: the forward and backward passes of one
 * parameter set run on that set, whatever other calls do meanwhile, and
 * nothing shared is written or synchronised).  d_arrhenius: 3*Nr doubles on
 * the device, [ln A (Nr), b (Nr), Ea/R (Nr)] in the description's reaction
 * order, the same meaning as pj_mech_set_arrhenius; read only, owned by the
 * caller, and it must stay valid until the call's work on `stream` is done.
 * NULL gives PJ_E_INVALID.  Everything else as pj_eval_source /
 * pj_eval_adjoint.
 */
pj_status pj_eval_source_arrhenius(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                                   const double* d_state, const double* d_param, const double* d_arrhenius,
                                   double* d_dstate, pj_stream stream);
pj_status pj_eval_adjoint_arrhenius(const pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                                    const double* d_state, const double* d_param, const double* d_arrhenius,
                                    const double* d_v, double* d_jtv, double* d_grad_or_null,
                                    double* d_dstate_or_null, pj_stream stream);

/*
 * Replace / read the Arrhenius parameters (ln A, b, Ea/R of k_f; of k_inf
 * for falloff and chemically activated reactions; of the factor on the
 * tabulated rate for P-Log and Chebyshev) of all Nr reactions, host arrays in description
 * order; a NULL array is left unchanged / not written.  Setting updates the
 * uploaded tables synchronously (the caller orders it against work in
 * flight that uses the mechanism).
 */
pj_status pj_mech_set_arrhenius(pj_mech* mech, const double* lnA, const double* b, const double* theta);
pj_status pj_mech_get_arrhenius(const pj_mech* mech, double* lnA, double* b, double* theta);

/*
 * Launch shape.  A workgroup evaluates states_per_group consecutive states at
 * once (a power of two up to 64) with waves_per_group waves (1 to 8); 1 state
 * per workgroup is the paper's deep mapping (Sec. 2.1: the lanes of a
 * workgroup cooperate on one state), 64 states on one wave its shallow
 * mapping (a lane per state).  0 restores the automatic choice (the most
 * states, up to 4, whose working set fits the LDS of one workgroup, and
 * enough waves for about 8 resident waves per compute unit).  A
 * states_per_group that does not fit for a mode is ignored for that mode.
 * With one wave per workgroup every accumulation happens in a fixed order,
 * so results are bitwise reproducible; with more, the order of LDS atomic
 * additions across waves may vary between runs (results then agree to
 * rounding).  pj_mech_set_waves_per_state(w) is pj_mech_set_launch(1, w)
 * (w in 1, 2, 4; 0 = automatic).
 */
pj_status pj_mech_set_launch(pj_mech* mech, int states_per_group, int waves_per_group);
pj_status pj_mech_set_waves_per_state(pj_mech* mech, int waves_per_state);
/* waves per workgroup when one state per workgroup is used, else -1 */
int pj_mech_waves_per_state(const pj_mech* mech, int for_jacobian);
/* launch shape of mode 0 (source), 1 (sparse Jacobian), 2 (dense Jacobian) or
 * 3 (adjoint, at most 4 states per workgroup); -1 on error */
int pj_mech_launch_shape(const pj_mech* mech, int mode, int* states_per_group, int* waves_per_group);

/*
 * The dense Jacobian's output loop reads the (row, column) -> CSR slot map of
 * the entries it writes with `entries` reads in flight per lane: 16 (the
 * default; 0 selects it) pays where a lane writes many entries, 8 where it
 * writes few (small mechanisms, many states per workgroup); 16 applies at up
 * to 4 states per workgroup, larger shapes read 8.  The autotuner of mode 2
 * chooses it with the shape.  The values are identical either way.
 * PJ_E_INVALID for NULL or another value; pj_mech_dense_unroll: the current
 * choice, -1 for NULL.
 */
pj_status pj_mech_set_dense_unroll(pj_mech* mech, int entries);
int pj_mech_dense_unroll(const pj_mech* mech);

/*
 * Autotuner: time every launch shape that fits (states per workgroup 1, 2,
 * 4, ..., 64; waves per workgroup 1 to 8; for mode 2 also the output loop's
 * 8 or 16 map reads in flight, pj_mech_set_dense_unroll) for mode 0
 * (source), 1 (sparse Jacobian) or 2 (dense Jacobian) on the caller's batch,
 * and keep the fastest for that mode until the next pj_mech_set_launch.  The buffers are those of
 * the matching evaluation call (d_out: d_dstate for mode 0, the Jacobian
 * output otherwise; d_dstate_or_null: the fused source output of modes 1 and
 * 2) and are overwritten.  Every shape runs one warm-up launch and `reps`
 * (>= 1) timed launches on `stream`; the call synchronises the stream.  On
 * success the chosen shape and its mean time per launch (ms) are stored
 * through the pointers that are not NULL.  Errors as for the evaluation
 * calls; PJ_E_INVALID also for a bad mode, reps < 1 or n_states < 1.
 */
pj_status pj_mech_autotune(pj_mech* mech, int mode, pj_form form, pj_layout layout, int64_t n_states,
                           const double* d_state, const double* d_param, double* d_out,
                           double* d_dstate_or_null, int reps, pj_stream stream,
                           int* states_per_group, int* waves_per_group, float* ms);

/* The autotuner for pj_eval_adjoint (states per workgroup at most 4), with
 * that call's buffers, which it overwrites. */
pj_status pj_mech_autotune_adjoint(pj_mech* mech, pj_form form, pj_layout layout, int64_t n_states,
                                   const double* d_state, const double* d_param, const double* d_v,
                                   double* d_jtv, double* d_grad_or_null, int reps, pj_stream stream,
                                   int* states_per_group, int* waves_per_group, float* ms);

/* Bytes of LDS one workgroup needs for source terms (0) or the sparse Jacobian (1). */
int64_t pj_mech_lds_bytes(const pj_mech* mech, int for_jacobian);

/*
 * Ragged multi-mechanism batches: segments of states of different mechanisms
 * (all uploaded on one device) evaluated by one persistent launch whose
 * workgroups take groups of states of any segment; the launch can be
 * captured once into a HIP graph and replayed.  Modes: 0 source terms
 * (d_out unused, source terms into d_dstate), 1 sparse Jacobian (d_out: CSR
 * values, d_dstate optional fused source terms), 3 adjoint (d_out: J^T v,
 * d_v required, d_grad optional 3*Nr parameter sums of that segment).
 * Buffers are caller-owned device memory in the layout given at evaluation,
 * and must stay valid while the batch (or its graph) may run.  The launch
 * shape S x W (S states per workgroup, a power of two up to 16, the adjoint
 * at most 4; W waves, 1 to 8) sets the LDS a workgroup gets: that of the
 * largest working set among the segments at S states.  Each segment then
 * takes the most states per workgroup (S doubled, up to 16; the adjoint up
 * to 4) whose working set fits that LDS (pj_batch_segment_states; -1 for a
 * NULL batch, a bad mode or segment index), so that segments of smaller
 * mechanisms hold more states at once.  Per mode, the batch can instead run
 * one launch per segment, each at its mechanism's own launch shape for that
 * mode (pj_batch_set_strategy(batch, mode, 1); 0 = the persistent launch,
 * the default); the graph then holds those launches.
 *
 * pj_batch_add records a segment (n_states may be 0); adding or clearing
 * segments, or changing the launch shape, discards a captured graph.
 * pj_batch_eval enqueues the batch on `stream` (the first call for a launch
 * shape uploads a small segment table synchronously).  pj_batch_eval_graph
 * captures the same work once per (mode, form, layout, shape) on a private
 * stream and launches the graph on `stream`; later calls replay it.
 * pj_batch_autotune times every fitting shape (as pj_mech_autotune) and one
 * launch per segment (at the mechanisms' current shapes), and keeps the
 * fastest for that mode: *states_per_group and *waves_per_group receive 0
 * when the per-segment launches win (the best persistent shape is kept as
 * the mode's launch shape either way).  pj_batch_strategy returns the mode's
 * strategy (0 or 1; -1 for a NULL batch or a bad mode).  Errors as for the
 * per-mechanism calls, with the segment index in the message
 * (pj_batch_last_error).
 */
typedef struct pj_batch pj_batch; /* opaque, library-owned */
pj_status pj_batch_create(pj_batch** out);
void pj_batch_free(pj_batch* batch); /* NULL-safe */
pj_status pj_batch_add(pj_batch* batch, const pj_mech* mech, int64_t n_states, const double* d_state,
                       const double* d_param, double* d_out, double* d_dstate_or_null,
                       const double* d_v_or_null, double* d_grad_or_null);
pj_status pj_batch_clear(pj_batch* batch);
int pj_batch_size(const pj_batch* batch); /* segments, -1 for NULL */
pj_status pj_batch_set_launch(pj_batch* batch, int mode, int states_per_group, int waves_per_group);
int pj_batch_launch_shape(const pj_batch* batch, int mode, int* states_per_group, int* waves_per_group);
int pj_batch_segment_states(const pj_batch* batch, int mode, int segment);
pj_status pj_batch_set_strategy(pj_batch* batch, int mode, int per_segment);
int pj_batch_strategy(const pj_batch* batch, int mode);
pj_status pj_batch_eval(pj_batch* batch, int mode, pj_form form, pj_layout layout, pj_stream stream);
pj_status pj_batch_eval_graph(pj_batch* batch, int mode, pj_form form, pj_layout layout, pj_stream stream);
/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid it): the batch's
 * persistent launch (whatever pj_batch_set_strategy says) with its segment
 * table in a fixed device array of the library, at most 64 non-empty
 * segments (PJ_E_UNSUPPORTED beyond), instead of device memory allocated
 * on the first call.  No hipMalloc, hipFree or allocating library call:
 * the table is written by a stream-ordered copy on `stream`, then the
 * launch.  Every call on one device shares that device's array, which keeps
 * the last call's table: calls that may overlap on one device (on different
 * streams, or from different threads) race; calls on one stream do not.
 * Outputs, modes, shapes and errors as pj_batch_eval.
 */
pj_status pj_batch_eval_noalloc(pj_batch* batch, int mode, pj_form form, pj_layout layout, pj_stream stream);
pj_status pj_batch_autotune(pj_batch* batch, int mode, pj_form form, pj_layout layout, int reps,
                            pj_stream stream, int* states_per_group, int* waves_per_group, float* ms);
const char* pj_batch_last_error(void);

/* Thread-local description of the last error ("" if none). */
const char* pj_last_error(void);

/*
 * Calibration of the FP64 operation weights of the device's own exp (fn 0),
 * log (1) and log10 (2), or of the loop alone (3): d_out[i] = sum over
 * r < reps of f(d_in[i] + r 1e-3), n values on `stream` (device arrays of n
 * doubles, caller-owned).  Profiling the four launches with the hardware's
 * FP64 counters gives the arithmetic one call of each function executes,
 * which weights the transcendentals in the source terms' operation count
 * (the FP64 roofline of Sec. 3.5.1's source-term timings).  PJ_E_INVALID
 * for a bad fn, n < 0, reps < 1 or NULL arrays; PJ_E_DEVICE if the launch
 * fails.
 */
pj_status pj_calibrate_fp64(int fn, int64_t n, int reps, const double* d_in, double* d_out, pj_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* PJAC_H */
