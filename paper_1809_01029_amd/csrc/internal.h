// Internal structures shared by the host mechanism compiler (mech.cpp), the
// kernels (kernel_body.h, kernels.hip, kernels_ext.hip) and the C-ABI (api.cpp,
// batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "pjac.h"

namespace pj {

constexpr double RU = 8314.462618;       // J/(kmol K)
constexpr double PREF = 101325.0;        // Pa
constexpr double LN10 = 2.302585092994045684;
constexpr int MAXSIDE = 3;               // species per reaction side
constexpr int NSLOT = 2 * MAXSIDE;       // reactant slots 0..2, product slots 3..5
constexpr uint16_t NOSLOT = 0xFFFF;
constexpr uint16_t DMAP_SKIP = 0xFFFE;   // dense map: entry written elsewhere

enum RxnKind : int { K_ELEM = 0, K_THREEBODY = 1, K_LINDEMANN = 2, K_TROE = 3, K_SRI = 4,
                     K_PLOG = 5, K_CHEB = 6 };
__host__ __device__ inline bool kind_falloff(int k) { return k >= K_LINDEMANN && k <= K_SRI; }
__host__ __device__ inline bool kind_table(int k) { return k == K_PLOG || k == K_CHEB; }
constexpr int MAX_PLOG = 64;          // pressures of one P-Log reaction
constexpr int MAX_CHEB = 16;          // Chebyshev coefficients per direction

// Bits of the per-reaction info word.
//   bits 0..23 : coefficient of slot a (a < 6) in bits 4a..4a+3 (0 = empty slot)
//   bits 24..26: kind (RxnKind)
//   bit  27    : reversible
//   bit  28    : the rate depends on the bath-gas concentration
//   bit  29    : the bath gas has a non-zero coefficient
//   bit  30    : chemically activated (falloff kinds)
constexpr uint32_t INFO_REV = 1u << 27;
constexpr uint32_t INFO_BATH = 1u << 28;
constexpr uint32_t INFO_BATHROW = 1u << 29;
constexpr uint32_t INFO_CHEMACT = 1u << 30;
constexpr uint32_t CHUNK_TAB = 1u << 12, CHUNK_SRI = 1u << 13, CHUNK_CHEMACT = 1u << 14;
__host__ __device__ inline int info_nu(uint32_t w, int a) { return (w >> (4 * a)) & 0xF; }
__host__ __device__ inline int info_kind(uint32_t w) { return (w >> 24) & 0x7; }

// Per-reaction device records, in the kernel order (sorted by kind) and
// padded to a multiple of 64 reactions.  Each record is 16-byte aligned and
// read with 16-byte vector loads.
struct alignas(16) RxnRec {          // 80 B
    uint32_t info;                   // see INFO_* above
    uint32_t eff;                    // index of this reaction's EffRec (third bodies; 0 = none)
    uint32_t neff;                   // number of third bodies with efficiency != 1
    uint32_t chunk;                  // slot positions used in this reaction's 64-reaction
                                     // chunk (bits 0..5), any reversible (bit 6), the
                                     // largest neff in the chunk (bits 8..11), any rate
                                     // tabulated in pressure (bit 12), any SRI (bit 13),
                                     // any chemically activated (bit 14)
    uint16_t sp[6];                  // species of slot a (Ns = empty slot)
    uint16_t tab;                    // P-Log / Chebyshev: index of the TabRec
    uint16_t pad1;
    double lnA, b, theta;            // Arrhenius (k_inf for falloff; a factor on a
                                     // rate tabulated in pressure)
    double dnu;                      // sum of net coefficients
    double domega;                   // sum_{k<Ns} nu_ki (1 - W_k/W_Ns)
    double bam1;                     // efficiency - 1 of the bath gas (0 if none)
};
struct alignas(16) FallRec {         // 64 B, falloff reactions
    double lnA0, b0, theta0;         // low-pressure limit
    double p[5];                     // Troe: alpha, 1/T***, 1/T*, T**
                                     // SRI:  a, b, 1/c, log10 d, e
};
struct alignas(16) TabRec {          // 48 B, rate constants tabulated in pressure
    int32_t off;                     // first double of the reaction's table
    int32_t n;                       // P-Log: pressures; Chebyshev: coefficients in T
    int32_t np;                      // Chebyshev: coefficients in P
    int32_t pad;
    double ta, tb;                   // Chebyshev: reduced temperature ta / T + tb
    double pa, pb;                   // Chebyshev: reduced pressure pa ln P + pb
};
// Table entries: P-Log, per pressure (ascending) {P, ln P, ln A, b, Ea/R, 0};
// Chebyshev, ln 10 * alpha_tp at t * np + p.
constexpr int PLOG_STRIDE = 6;
struct alignas(16) JacRec {          // 96 B, Jacobian scatter slots (NOSLOT = none)
    uint16_t rowbase[6];             // CSR start of the row of slot a's species
    uint16_t pad0[2];
    uint16_t slot[36];               // CSR slot of (row of slot a, column of slot b), [a*6+b]
    uint16_t pad1[4];
};
constexpr int MAXEFF = 8;             // third bodies with efficiency != 1 per reaction
struct alignas(16) EffRec {          // 176 B, third-body reactions; record 0 is
                                     // all-empty and serves the elementary ones
    uint16_t sp[MAXEFF];             // species (Ns = unused entry)
    double am1[MAXEFF];              // efficiency - 1
    uint16_t slot[6][MAXEFF];        // CSR slot of (row of reaction slot a, column of
                                     // entry e) at [a][e]
};
static_assert(sizeof(RxnRec) == 80 && sizeof(FallRec) == 64 && sizeof(JacRec) == 96 &&
              sizeof(EffRec) == 176 && sizeof(TabRec) == 48, "record sizes");

// Thermodynamic coefficients of one species and one temperature range.
constexpr int TH_N = 18;
struct alignas(16) ThermoRec {       // 144 B
    double c[TH_N];
};

// Device pointers held in the table and batch descriptors: in the device
// pass they are global-memory pointers, so that a descriptor read from
// device memory (a ragged batch's segment table), like a kernel argument,
// gives global rather than flat memory instructions; the host pass sees
// plain pointers of the same size and layout.
#if defined(__HIP_DEVICE_COMPILE__)
#define PJ_GLOBAL __attribute__((address_space(1)))
#else
#define PJ_GLOBAL
#endif
// a device pointer as stored in a descriptor
template <class T>
inline PJ_GLOBAL T* gptr(T* p) {
    return (PJ_GLOBAL T*)p;
}

struct DevMech {
    int ns, nr, nr_pad, N;
    int nnz;            // CSR non-zeros
    int n_dense_rows;   // species rows made dense by bath-gas dependent rates
    int bath;           // ns - 1

    // species
    const PJ_GLOBAL ThermoRec* th;      // [ns][2] (low range, high range)
    const PJ_GLOBAL double* tmid;       // [ns]
    const PJ_GLOBAL double* wfac;       // [ns] 1 - W_k / W_Ns (0 for the bath gas)

    // reactions
    const PJ_GLOBAL RxnRec* rec;        // [nr_pad]
    const PJ_GLOBAL FallRec* fall;      // [nr_pad]
    const PJ_GLOBAL JacRec* jrec;       // [nr_pad]
    const PJ_GLOBAL EffRec* effrec;     // [1 + reactions with third bodies]
    const PJ_GLOBAL TabRec* tab;        // [reactions tabulated in pressure, at least 1]
    const PJ_GLOBAL double* tabd;       // their tables

    // pattern
    const PJ_GLOBAL int32_t* row_ptr;   // [N + 1]
    const PJ_GLOBAL uint16_t* row_of;   // [nnz] row (state index) of each CSR entry
    const PJ_GLOBAL uint16_t* ccs_pos;  // [nnz] position of CSR entry e in column order, or NULL
    const PJ_GLOBAL uint16_t* dmap_rm;  // [N*N] CSR slot of (i, j) at i*N + j, NOSLOT if none
    const PJ_GLOBAL uint16_t* dmap_cm;  // [N*N] the same at i + N*j; DMAP_SKIP for rows 0 and 1
    int approx;               // approximate Jacobian (bath gas held against n_j)
    int ext;                  // holds SRI, chemically activated, P-Log or Chebyshev reactions
    int lsearch;              // find CSR slots by a run-time row search
    int det;                  // every LDS addition in a fixed order (bitwise reproducible)
    const PJ_GLOBAL int32_t* orig;      // [nr] description index of each kernel-order reaction
    const PJ_GLOBAL uint16_t* col_idx;  // [nnz]
    const PJ_GLOBAL int32_t* dense_rows;// [n_dense_rows] species index k of bath-dense rows
    const PJ_GLOBAL double* arr;        // NULL, or one call's Arrhenius parameters [ln A (nr), b (nr),
                              // Ea/R (nr)] in description order, in place of the tables
};

struct Mechanism {
    // host copy of the description
    int ns = 0, nr = 0;
    std::vector<double> W;
    std::vector<int> comp;                 // [ns][4]
    std::vector<double> tmid, alo, ahi;    // alo/ahi: [ns][7]
    struct Rxn {
        int kind;
        bool rev;
        std::vector<std::pair<int, int>> reac, prod;
        double lnA, b, theta;
        double lnA0 = 0, b0 = 0, theta0 = 0;
        double alpha = 0, T3 = 1, T1 = 1, T2 = 0;
        double sri[5] = {0, 0, 0, 0, 0};   // a, b, c, d, e
        bool chemact = false;
        std::vector<std::pair<int, double>> eff;
        std::vector<std::array<double, 4>> plog;   // (P, ln A, b, Ea/R), ascending P
        int cheb_nt = 0, cheb_np = 0;
        double cheb_T[2] = {0, 0}, cheb_P[2] = {0, 0};
        std::vector<double> cheb;                  // [nt][np]
    };
    std::vector<Rxn> rx;

    int opts = 0;                          // PJ_OPT_* given at parse time
    // derived
    std::vector<int> order;                // kernel position -> description index
    std::vector<int32_t> row_ptr, col_idx; // CSR pattern
    std::vector<int32_t> col_ptr, row_idx; // the same pattern in column order (CCS)
    int nnz = 0;

    // device
    int device = -1;
    void* dbuf = nullptr;
    DevMech dm{};
    // launch shape per mode (source, sparse, dense): states per workgroup,
    // waves per workgroup, and the LDS bytes that needs
    int S[4] = {1, 1, 1, 1}, waves[4] = {1, 1, 1, 1};
    int64_t lds[4] = {0, 0, 0, 0};
    bool adj_grad_in_lds = true;           // adjoint parameter sums kept in LDS
    // host copy of the reaction records and their byte offset in the device
    // buffer (Arrhenius parameters can be replaced after the upload)
    std::vector<RxnRec> h_rec;
    size_t off_rec = 0;
    int user_S = 0, user_waves = 0;        // 0 = automatic
    int dense_unroll = 16;                 // dense output: map entries in flight per lane (8 or 16)
    int lds_max = 0;
};

// One segment of a ragged multi-mechanism batch, as the batch kernel reads
// it from device memory.
struct BatchSeg {
    DevMech dm;
    long n;                    // states of this segment
    const PJ_GLOBAL double* state;
    const PJ_GLOBAL double* param;
    PJ_GLOBAL double* dstate;            // source terms (source mode) or fused source output
    PJ_GLOBAL double* out;               // CSR values (sparse) or J^T v (adjoint)
    const PJ_GLOBAL double* vin;         // adjoint: v
    PJ_GLOBAL double* grad;              // adjoint: parameter sums (3 Nr) or NULL
    long g0;                   // first global group index of this segment
    int S;                     // states per group of this segment (1 to 16, a power of two)
    long gr_off;               // adjoint: LDS offset (doubles) of its parameter sums, or -1
};

// The most states per group a segment of a ragged batch takes (the adjoint:
// MAX_S_ADJ): segments of smaller mechanisms fill the workgroup LDS that the
// largest mechanism's states set with more states each.
constexpr int BATCH_MAX_S = 16;

// mech.cpp
pj_status build_mechanism(const char* path, Mechanism& m, std::string& err);
pj_status upload_mechanism(Mechanism& m, std::string& err);

// kernels.hip (kernel_body.h)
enum Mode : int { MODE_SRC = 0, MODE_SPARSE = 1, MODE_DENSE = 2, MODE_ADJ = 3,
                  MODE_SPARSE_LS = 4 /* sparse with run-time slot search; launch shape of MODE_SPARSE */,
                  // source terms / adjoint with the call's own Arrhenius parameters
                  // (DevMech::arr); launch shapes of MODE_SRC / MODE_ADJ
                  MODE_SRC_P = 5, MODE_ADJ_P = 6,
                  // source terms / sparse Jacobian with every LDS addition in a fixed
                  // order (the waves of a workgroup add in turn); shapes of MODE_SRC /
                  // MODE_SPARSE, at most 4 states per workgroup
                  MODE_SRC_DET = 7, MODE_SPARSE_DET = 8,
                  // dense Jacobian writing its output with 16 map entries in flight
                  // per lane instead of 8; launch shape of MODE_DENSE, at most 4
                  // states per workgroup (more keep 8)
                  MODE_DENSE_U16 = 9 };
// the mode whose computation a kernel mode performs
__host__ __device__ constexpr int base_mode(int m) {
    return m == MODE_SRC_P || m == MODE_SRC_DET ? MODE_SRC
           : m == MODE_ADJ_P ? MODE_ADJ : m == MODE_SPARSE_DET ? MODE_SPARSE
           : m == MODE_DENSE_U16 ? MODE_DENSE : m;
}
constexpr int N_MODES = 4;        // modes with a launch shape of their own
constexpr int MAX_S_ADJ = 4;      // states per workgroup of the adjoint mode
// grad_in_lds: the adjoint keeps its parameter sums in LDS (mode MODE_ADJ only)
int64_t lds_bytes(const DevMech& dm, int mode, int S, int waves, bool grad_in_lds = true);
hipError_t launch(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                  const double* state, const double* param, double* dstate, double* jac,
                  const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                  hipStream_t stream);
hipError_t zero_async(double* p, int64_t n, hipStream_t stream);
// batch kernel (modes source, sparse, adjoint; each segment's states per
// group and adjoint parameter-sum placement in its table entry)
// ext: some segment's mechanism holds the further reaction types
// su: the states per group every segment takes (1, 2 or 4: a compile-time
// group body), or 0 (each segment's own, read at run time)
hipError_t launch_batch(int mode, int form, int layout, int waves, int64_t lds, const BatchSeg* d_segs,
                        int nseg, int64_t total_groups, int ext, int su, hipStream_t stream);
// kernels_conv.hip, kernels_ext.hip, kernels_ext_conv.hip: the same launches
// for the CONV form, for mechanisms with the further reaction types (CONP),
// and for both (CONV)
hipError_t launch_conv(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                       const double* state, const double* param, double* dstate, double* jac,
                       const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                       hipStream_t stream);
hipError_t launch_ext_conv(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                           const double* state, const double* param, double* dstate, double* jac,
                           const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                           hipStream_t stream);
hipError_t launch_ext(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                      const double* state, const double* param, double* dstate, double* jac,
                      const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                      hipStream_t stream);
hipError_t launch_batch_ext(int mode, int form, int layout, int waves, int64_t lds, const BatchSeg* d_segs,
                            int nseg, int64_t total_groups, int su, hipStream_t stream);
// api.cpp
void choose_launch(Mechanism& m);

}  // namespace pj

struct pj_mech {
    pj::Mechanism m;
};

namespace pj {
// noalloc.hip: most segments pj_batch_eval_noalloc takes
constexpr int NOALLOC_MAX_SEGS = 64;
}  // namespace pj

// A ragged multi-mechanism batch (batch.cpp, noalloc.hip).
struct pj_batch {
    struct Seg {
        const pj_mech* mech;
        int64_t n;
        const double* state;
        const double* param;
        double* out;
        double* dstate;
        const double* v;
        double* grad;
    };
    std::vector<Seg> segs;
    int device = -1;
    int user_S[pj::N_MODES] = {0, 0, 0, 0}, user_W[pj::N_MODES] = {0, 0, 0, 0};
    int per_seg[pj::N_MODES] = {0, 0, 0, 0};   // 1: one launch per segment
    // device copy of the segment table, for the shape it was built with
    pj::BatchSeg* d_segs = nullptr;
    size_t d_cap = 0;
    int table_S = 0, table_W = 0, table_mode = -1, table_nseg = 0;
    int64_t table_total = 0;
    bool table_valid = false;
    // captured graph and what it was captured for
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_mode = -1, g_form = -1, g_layout = -1, g_S = 0, g_W = 0, g_per_seg = 0;
    hipStream_t capture_stream = nullptr;
    // host staging of pj_batch_eval_noalloc's segment table
    pj::BatchSeg noalloc_host[pj::NOALLOC_MAX_SEGS] = {};

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        g_mode = -1;
    }
};

namespace pj {
// batch.cpp: the batch's argument checks, launch shape and LDS size, and its
// error message (pj_batch_last_error)
pj_status batch_fail(pj_status st, const std::string& msg);
void batch_ok();
pj_status batch_check(const pj_batch* b, int mode, pj_form form, pj_layout layout);
void batch_shape_of(const pj_batch* b, int mode, int& S, int& W);
// the LDS the batch needs at S x W, and its launch's LDS per workgroup
int64_t batch_lds_of(const pj_batch* b, int mode, int S, int W);
int64_t batch_launch_lds(const pj_batch* b, int mode, int S, int W);
// the persistent launch's segment table at S x W into t (room for cap
// entries): the entry count (-1 beyond cap), the groups of all in *total,
// whether a mechanism needs the further reaction types' kernels in *ext
int batch_fill_table(const pj_batch* b, int mode, int S, int W, BatchSeg* t, int cap, long* total, int* ext);
// the states per group all non-empty segments share at S x W when it is 1, 2
// or 4 (the batch kernel then has a compile-time group body), else 0
int batch_uniform_states(const pj_batch* b, int mode, int S, int W);
int batch_lds_limit(const pj_batch* b);
}  // namespace pj
