// FP64 HIP kernels for gfx950: thermochemical source terms and the analytical
// sparse / dense Jacobian (Curtis, Niemeyer & Sung, pyJac v2, Sec. 2.2 and
// Sec. 3.4), with the lanes of a workgroup cooperating on a few states at a
// time ("deep" vectorization, Sec. 2.1).
//
// Mapping.  A workgroup evaluates S consecutive states at once (S = 1, 2, 4,
// ..., 64) in a grid-stride loop over groups of states.  Thread t works for
// state t mod S; the t / S index splits the species for the thermodynamics
// and the reactions (sorted by kind and shape) for the rates and the Jacobian
// sub-products, so the S lanes of one reaction fetch its record together.
// S = 1 is the "deep" mapping of the paper (Sec. 2.1: a workgroup cooperates
// on one state); S = 64 with one wave is its "shallow" mapping (each lane owns
// a state and walks all reactions, reading every table entry as a wave-wide
// broadcast); the sizes between trade LDS per workgroup for fewer lanes per
// state.
// The per-state working set lives in LDS, every array interleaved with the
// state fastest (element i of state s at i*S + s):
//     C, G, H, CP, W   [Ns+1] concentrations, g = G/RT, h = H/RT, chat/R,
//                      production rates; entry Ns is a sentinel (C = 1,
//                      G = H = 0) that empty reaction slots point at
//     J                [nnz]  CSR accumulator of the species rows (the
//                      adjoint: only the 2N slots of TQ and SQ)
//     B                [Ns]   per-row sum of the bath-gas partials
//     TQ, SQ           [Ns+1] energy- and mole-weighted concentration
//                      partials, kept in the space of CSR rows 0 and 1 (the
//                      finished T and V/P rows are staged in the G and H
//                      arrays and written out with the species rows)
//     VV, JTV          [N], [N+2] (adjoint) the vector v and J^T v (two
//                      entries past N catch the bath gas's and empty slots'
//                      terms)
//     GR               [3 Nr] (adjoint, per workgroup, not per state) the
//                      workgroup's sums of the Arrhenius-parameter derivatives
// Reactions scatter into these with LDS FP64 atomics (ds_add_f64).  Because
// the S states of one reaction sit in adjacent words, one atomic instruction
// touches 64/S reactions in S-word blocks; the order of the species within a
// reaction side is chosen per 64-reaction chunk so that hub species do not
// repeat one address within an instruction.  With one wave per workgroup the
// order of those additions is fixed by program order, so results are bitwise
// reproducible.
//
// Jacobian formulation.  With the third-body concentration written as
// [M] = C_tot + sum_k (alpha_k - 1) [C]_k, C_tot = P/(R T), each reaction
// provides Q_j = dq/d[C]_j at fixed T and C_tot, Q_M = dq/dC_tot, and
// dq/dT at fixed concentrations.  The bath-gas closure then gives
//     dq/dn_j = (Q_j - Q_Ns) / V,   dq/dT = q_T - C_tot/T (Q_Ns + Q_M),
//     CONP  dq/dV = -(sum_{j<Ns} Q_j [C]_j - Q_Ns sum_{j<Ns} [C]_j) / V,
//     CONV  dq/dP = (Q_Ns + Q_M) / (R T),
// so species row k of J holds sum_i nu_ki (Q_ij - Q_iNs) in its species
// columns and V sum_i nu_ki dq_i/dx in the T and V/P columns.  The T row
// follows from differentiating dT/dt = -N/D and the V/P row from the ideal-gas
// form of dV/dt or dP/dt; both need sum_i dE_i Q_ij and sum_i dOmega_i Q_ij,
// accumulated in TQ and SQ.
//
// Adjoint.  J^T v is formed without the Jacobian: reaction i enters species
// row k only as nu_ki times the gradient of q_i, so its part of v^T J is
// vn_i grad q_i with vn_i = sum_k nu_ki v_k over its species rows.  It adds
// vn_i Q_ij to column j (third bodies: vn_i Q_M (alpha_j - 1)), and per-thread
// sums of vn_i V dq_i/dT, vn_i V dq_i/dS (the species rows' T and V/P
// columns) and vn_i Q_iNs (the bath partial the dense rows take out of every
// species column) are reduced with the source terms; the T and V/P rows then
// add v_T J_0j + v_S J_1j to every column, and CONP adds sum_k v_k wdot_k to
// the V column (d(V wdot_k)/dV = wdot_k + V dwdot_k/dV).  The
// Arrhenius-parameter derivatives of v . dPhi/dt use that the source terms
// depend on reaction i's parameters only through q_i:
//     d(v . f)/d theta_i = lambda_i dq_i/d theta_i,
//     lambda_i = v_T dTdot/dq_i + v_S dSdot/dq_i + V sum_k v_k nu_ki,
//     dTdot/dq_i = -T dE_i / D',  CONP dSdot/dq_i = V/T dTdot/dq_i + V R T/P dOmega_i,
//     CONV dSdot/dq_i = P/T dTdot/dq_i + R T dOmega_i,
//     dq_i/d ln A = q_i - (Rf - Rr) Pr dc/dPr (falloff forms; q_i otherwise),
//     dq_i/db = ln T dq_i/d ln A,  dq_i/d(Ea/R) = -dq_i/d ln A / T.
//
// Reaction types.  Elementary; third-body; falloff with the Lindemann, Troe
// or SRI broadening F(Pr, T); chemically activated with the same forms; rate
// constants tabulated in pressure (P-Log, Chebyshev).  The rate of progress
// always carries the main Arrhenius expression: k_inf for the falloff forms
// (a chemically activated reaction's c = F k0 / (k_inf (1 + Pr)) then turns
// it into k0 F / (1 + Pr)), and a factor on the tabulated k for P-Log and
// Chebyshev, whose d ln k/dP enters dq/dP, the P column of the constant-
// volume form.  With Pr dc/dPr taken at fixed [M], dq/d ln A above holds for
// every type.
//
// This header holds the kernels as templates; kernels.hip instantiates them
// for mechanisms of the default reaction types, kernels_ext.hip for the
// mechanisms that also hold the further types (EXT = true), so that the two
// sets compile in parallel and the default kernels carry none of the further
// types' code.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>

#include "internal.h"

namespace pj {


namespace {

// LDS scratch of the workgroup reductions, per state and wave: up to 10
// values; the last entry of the area (never reached by a reduction) holds the
// reaction loop's block counter
constexpr int RED_PER_WAVE = 11;
constexpr int MAX_THREADS = 512;
// s_waitcnt lgkmcnt(0) (vmcnt and expcnt at their maxima, gfx9 encoding)
constexpr int WAIT_LGKM0 = 0xC07F;

struct dd {
    double hi, lo;
};

// Error-free transformations (Knuth TwoSum, Dekker FastTwoSum)
__device__ inline void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ inline void fast_two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    e = b - (s - a);
}
// double-double addition (accurate variant)
__device__ inline dd dd_add(dd a, dd b) {
    double s, t, u, v;
    two_sum(a.hi, b.hi, s, t);
    two_sum(a.lo, b.lo, u, v);
    t += u;
    fast_two_sum(s, t, s, t);
    t += v;
    fast_two_sum(s, t, s, t);
    return {s, t};
}

// Sum over the lanes of a wave that work for the same state (lanes equal
// modulo S); every such lane receives the sum.
template <int S>
__device__ inline double wave_sum(double v, int Sr = S) {
    if constexpr (S > 0) {
#pragma unroll
        for (int o = 32; o >= S; o >>= 1) v += __shfl_xor(v, o, 64);
    } else {
        for (int o = 32; o >= Sr; o >>= 1) v += __shfl_xor(v, o, 64);
    }
    return v;
}

// Per-state sum of K per-thread values over the workgroup, in a fixed order;
// every thread receives the totals of its state.  red: LDS scratch of
// RED_PER_WAVE * nwave * S doubles.  S = 0: Sr states per group, known at
// run time.
template <int S, int K>
__device__ inline void block_sum(double (&v)[K], double* red, int wave, int nwave, int s, int Sr = S) {
    static_assert(K <= RED_PER_WAVE - 1, "reduction scratch per wave");
    const int SR = S > 0 ? S : Sr;
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = wave_sum<S>(v[q], SR);
    if (nwave == 1) return;
    if ((threadIdx.x & 63) < SR) {
#pragma unroll
        for (int q = 0; q < K; ++q) red[(wave * K + q) * SR + s] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double t = 0.0;
        for (int w = 0; w < nwave; ++w) t += red[(w * K + q) * SR + s];
        v[q] = t;
    }
    __syncthreads();
}

template <int S>
__device__ inline dd block_dd_sum(dd a, double* red, int wave, int nwave, int s, int Sr = S) {
    const int SR = S > 0 ? S : Sr;
    auto step = [&](int o) {
        dd b{__shfl_xor(a.hi, o, 64), __shfl_xor(a.lo, o, 64)};
        a = dd_add(a, b);
    };
    if constexpr (S > 0) {
#pragma unroll
        for (int o = 32; o >= S; o >>= 1) step(o);
    } else {
        for (int o = 32; o >= SR; o >>= 1) step(o);
    }
    if (nwave == 1) return a;
    if ((threadIdx.x & 63) < SR) {
        red[(2 * wave) * SR + s] = a.hi;
        red[(2 * wave + 1) * SR + s] = a.lo;
    }
    __syncthreads();
    dd t{0.0, 0.0};
    for (int w = 0; w < nwave; ++w) t = dd_add(t, dd{red[(2 * w) * SR + s], red[(2 * w + 1) * SR + s]});
    __syncthreads();
    return t;
}

// 16-byte vector loads of a table record
template <class T>
__device__ inline T load_rec(const PJ_GLOBAL T* src) {
    static_assert(sizeof(T) % 16 == 0, "record size");
    union U {
        T t;
        uint4 v[sizeof(T) / 16];
    } u;
    const PJ_GLOBAL uint4* q = (const PJ_GLOBAL uint4*)src;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 16); ++i) u.v[i] = q[i];
    return u.t;
}

// ln k of a rate constant tabulated in pressure, with its partial derivatives
// by T (at fixed P) and by P (at fixed T).
//   P-Log: between the two tabulated pressures that bracket P, ln k is linear
//   in ln P (each pressure has its own Arrhenius expression); below the first
//   and above the last pressure that end's expression holds.
//   Chebyshev: ln k = ln 10 sum_t sum_p alpha_tp T_t(Tr) T_p(Pr), Tr and Pr the
//   reduced inverse temperature and log pressure, the polynomials and their
//   derivatives from the three-term recurrence.
__device__ inline double table_lnk(const DevMech& dm, int kind, int ti, double T, double invT,
                                   double lnT, double P, double& dT, double& dP) {
    const TabRec tr = load_rec(dm.tab + ti);
    const double* d = dm.tabd + tr.off;
    if (kind == K_PLOG) {
        auto at = [&](int i, double& di) {
            const double* e = d + (size_t)i * PLOG_STRIDE;
            const double b = e[3], th = e[4];
            di = (b + th * invT) * invT;
            return e[2] + b * lnT - th * invT;
        };
        const int n = tr.n;
        dP = 0.0;
        if (!(P > d[0])) return at(0, dT);
        if (!(P < d[(size_t)(n - 1) * PLOG_STRIDE])) return at(n - 1, dT);
        int i = 0;   // P_0 < P < P_{n-1}: find P_i <= P < P_{i+1}
        while (P >= d[(size_t)(i + 1) * PLOG_STRIDE]) ++i;
        double d1, d2;
        const double l1 = at(i, d1), l2 = at(i + 1, d2);
        const double lp1 = d[(size_t)i * PLOG_STRIDE + 1], lp2 = d[(size_t)(i + 1) * PLOG_STRIDE + 1];
        const double lnP = log(P);
        const double slope = (l2 - l1) / (lp2 - lp1);
        const double w = (lnP - lp1) / (lp2 - lp1);
        dT = d1 + w * (d2 - d1);
        dP = slope / P;
        return l1 + slope * (lnP - lp1);
    }
    const double Tr = tr.ta * invT + tr.tb;
    const double Pr = tr.pa * log(P) + tr.pb;
    double v = 0.0, vT = 0.0, vP = 0.0;
    double t0 = 1.0, t1 = Tr, dt0 = 0.0, dt1 = 1.0;   // T_t(Tr), T_{t+1}(Tr) and derivatives
    for (int t = 0; t < tr.n; ++t) {
        double s = 0.0, sd = 0.0;
        double p0 = 1.0, p1 = Pr, dp0 = 0.0, dp1 = 1.0;
        for (int q = 0; q < tr.np; ++q) {
            const double a = d[t * tr.np + q];
            s += a * p0;
            sd += a * dp0;
            const double p2 = 2.0 * Pr * p1 - p0, dp2 = 2.0 * p1 + 2.0 * Pr * dp1 - dp0;
            p0 = p1;
            p1 = p2;
            dp0 = dp1;
            dp1 = dp2;
        }
        v += s * t0;
        vT += s * dt0;
        vP += sd * t0;
        const double t2 = 2.0 * Tr * t1 - t0, dt2 = 2.0 * t1 + 2.0 * Tr * dt1 - dt0;
        t0 = t1;
        t1 = t2;
        dt0 = dt1;
        dt1 = dt2;
    }
    dT = -vT * tr.ta * invT * invT;
    dP = vP * tr.pa / P;
    return v;
}

// Species (two 16-bit entries per word) and efficiency - 1 of the first
// n (uniform over the wave) third bodies of a reaction; the rest read as 0
__device__ inline void load_eff(const EffRec* r, int n, uint32_t (&sp)[MAXEFF / 2],
                                double (&am1)[MAXEFF]) {
    const uint4* q = reinterpret_cast<const uint4*>(r);
    const uint4 v = q[0];
    sp[0] = v.x;
    sp[1] = v.y;
    sp[2] = v.z;
    sp[3] = v.w;
#pragma unroll
    for (int h = 0; h < MAXEFF / 2; ++h) {
        if (2 * h < n) {
            const uint4 u = q[1 + h];
            am1[2 * h] = __hiloint2double(u.y, u.x);
            am1[2 * h + 1] = __hiloint2double(u.w, u.z);
        } else {
            am1[2 * h] = am1[2 * h + 1] = 0.0;
        }
    }
}
__device__ inline int eff_species(const uint32_t (&sp)[MAXEFF / 2], int e) {
    return (sp[e >> 1] >> (16 * (e & 1))) & 0xFFFF;
}

// CSR slot of (row, col) by a search of the row (the run-time lookup the
// static slot map replaces; used only when the mechanism asks for it)
__device__ inline uint16_t csr_lookup(const DevMech& dm, int row, int col) {
    const int r0 = dm.row_ptr[row], r1 = dm.row_ptr[row + 1];
    for (int e = r0; e < r1; ++e)
        if (dm.col_idx[e] == col) return (uint16_t)e;
    return NOSLOT;
}

// c^nu and d(c^nu)/dc for nu in {0, 1, 2} with selects instead of branches;
// an empty slot (nu = 0) reads the sentinel concentration 1, giving f = 1
__device__ inline void powd(double c, int nu, double& f, double& d) {
    f = nu == 2 ? c * c : c;
    d = nu == 2 ? 2.0 * c : (double)nu;
}

}  // namespace

// One group of S consecutive states (group index qg of a batch of n): the
// body shared by the per-mechanism kernel and the ragged multi-mechanism
// kernel.  S = 0: Sr states per group, given at run time (the ragged kernel,
// whose segments each have their own).  GR / gr_lds: the adjoint's
// per-workgroup parameter sums in LDS (or per-group device atomics when
// gr_lds is false).
template <int FORM, int LAYOUT, int MODE, int S, bool EXT>
__device__ __forceinline__ void eval_group(const DevMech& dm, const long n,
                                           const double* __restrict__ state,
                                           const double* __restrict__ param,
                                           double* __restrict__ dstate,
                                           double* __restrict__ jac,
                                           const double* __restrict__ vin,
                                           double* __restrict__ grad,
                                           const bool gr_lds, double* GR, const long qg,
                                           const int Sr = S) {
    extern __shared__ double lds[];
    // states per group: S, or Sr (a power of two, 1 to 16) when S = 0;
    // LG = log2 of it (indexing by shifts also when it is known at run time)
    const int SR = S > 0 ? S : Sr;
    const int LG = __builtin_ctz((unsigned)SR);
    constexpr int M = base_mode(MODE);
    constexpr bool PAR = MODE == MODE_SRC_P || MODE == MODE_ADJ_P;   // the call's own Arrhenius parameters
    constexpr bool DET = MODE == MODE_SRC_DET || MODE == MODE_SPARSE_DET;   // additions in a fixed order
    constexpr bool JAC = M != MODE_SRC;
    constexpr bool ADJ = M == MODE_ADJ;      // jac receives J^T v (state layout)
    constexpr bool LS = M == MODE_SPARSE_LS;   // sparse, slots found by a row search
    constexpr bool SPARSE = M == MODE_SPARSE || LS;
    const int ns = dm.ns, N = dm.N, bath = dm.bath, nnz = dm.nnz;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, nwave = nthr >> 6;
    const int s = tid & (SR - 1);    // the state of this thread within the group
    const int g = tid >> LG;         // its index among the threads of that state
    const int G = nthr >> LG;        // threads per state

    double* C = lds;
    double* Gg = C + (ns + 1) * SR;
    double* H = Gg + (ns + 1) * SR;
    double* CP = H + (ns + 1) * SR;
    double* W = CP + (ns + 1) * SR;
    double* red = W + (ns + 1) * SR;
    double* J = red + RED_PER_WAVE * nwave * SR;
    // the reaction loop's block counter: the last entry of the reduction area
    int* const bctr = reinterpret_cast<int*>(J - 1);
    // the adjoint forms J^T v without the Jacobian: of J it keeps the T and
    // V/P rows' partial sums only
    const int nj = ADJ ? 2 * N : nnz;
    // the sparse and dense kernels send the additions of row-column pairs
    // that do not exist to 64 sink entries past the accumulator (entry
    // nj + k for lane block k: 64/S per state), so that a scatter needs no
    // per-lane branch and no two lanes of an instruction meet at a sink
    constexpr int NSINK = JAC && !ADJ ? 64 : 0;
    double* B = J + (size_t)nj * SR + NSINK;
    double* VV = B + (size_t)ns * SR;      // adjoint: v
    double* JTV = VV + (size_t)N * SR;     // adjoint: J^T v (N + 2 entries, the last two never read)
    // The LDS of the T and V/P rows (the first 2N CSR slots) holds the
    // energy- and mole-weighted partial sums; the finished rows are staged
    // in the G and H arrays.
    double* TQ = J;
    double* SQ = J + (size_t)N * SR;
#define AT(arr, i) (arr)[((size_t)(i) << LG) + s]

    {
        const long st = qg * SR + s;           // this thread's state
        const bool valid = st < n;
        const long sc = valid ? st : n - 1;   // states past the end compute a copy of the last
        auto X = [&](int i) -> double {
            return LAYOUT == PJ_LAYOUT_F ? state[(long)i * n + sc] : state[sc * (long)N + i];
        };
        const double T = X(0);
        const double Sv = X(1);
        const double Q = param[sc];
        const double V = FORM == PJ_CONP ? Sv : Q;
        const double P = FORM == PJ_CONP ? Q : Sv;
        const double invT = 1.0 / T;
        const double invV = 1.0 / V;

        // ---- concentrations and the bath-gas closure (Sec. 2.2):
        //      n_Ns = P V / (R T) - RN(sum_{k<Ns} n_k)
        // the accumulators are cleared while the state's loads are in flight
        for (int k = g; k < ns + 1; k += G) AT(W, k) = 0.0;
        if (JAC && !DET && !ADJ && tid == 0) *bctr = 0;
        if (JAC) {
            for (int e = g; e < nj; e += G) AT(J, e) = 0.0;
            for (int k = g; k < ns; k += G) AT(B, k) = 0.0;
        }
        if (ADJ) for (int i = g; i < N + 2; i += G) AT(JTV, i) = 0.0;
        dd acc{0.0, 0.0};
        for (int k = g; k < ns - 1; k += G) {
            const double nk = X(2 + k);
            acc = dd_add(acc, dd{nk, 0.0});
            AT(C, k) = nk / V;
        }
        if (ADJ) {
            for (int i = g; i < N; i += G)
                AT(VV, i) = LAYOUT == PJ_LAYOUT_F ? vin[(long)i * n + sc] : vin[sc * (long)N + i];
        }
        acc = block_dd_sum<S>(acc, red, wave, nwave, s, SR);
        const double nsum = acc.hi;
        const double ntot = (P * V) / (RU * T);
        const double nbath = ntot - nsum;
        if (g == 0) {
            AT(C, bath) = nbath / V;
            AT(C, ns) = 1.0;
            AT(Gg, ns) = 0.0;
            AT(H, ns) = 0.0;
            AT(CP, ns) = 0.0;
        }
        __syncthreads();

        const double lnT = log(T);
        const double Ctot = P / (RU * T);
        const double lnP0RT = log(PREF / (RU * T));
        const double invRT = 1.0 / (RU * T);

        // ---- species thermodynamics (NASA-7)
        double tsum[2] = {0.0, 0.0};   // D' = sum C chat/R, dD'/dT = sum C dCp/R/dT
        for (int k = g; k < ns; k += G) {
            const int rg = T < dm.tmid[k] ? 0 : 1;
            const ThermoRec tr = load_rec(dm.th + 2 * (size_t)k + rg);
            auto a = [&](int q) { return tr.c[q]; };
            const double a0 = a(0), a1 = a(1);
            const double cp = a0 + T * (a1 + T * (a(2) + T * (a(3) + T * a(4))));
            const double h = a0 + T * (a(5) + T * (a(6) + T * (a(7) + T * a(8)))) + a(12) * invT;
            const double sr = a0 * lnT + T * (a1 + T * (a(9) + T * (a(10) + T * a(11)))) + a(13);
            AT(Gg, k) = h - sr;
            AT(H, k) = h;
            const double ch = FORM == PJ_CONP ? cp : cp - 1.0;
            AT(CP, k) = ch;
            const double ck = AT(C, k);
            tsum[0] += ck * ch;
            if (JAC) tsum[1] += ck * (a1 + T * (a(14) + T * (a(15) + T * a(16))));
        }
        block_sum<S>(tsum, red, wave, nwave, s, SR);
        const double Dp = tsum[0];
        const double dDpdT = tsum[1];
        __syncthreads();
        const double vT = ADJ ? AT(VV, 0) : 0.0, vS = ADJ ? AT(VV, 1) : 0.0;

        // ---- reactions: rates of progress and Jacobian sub-products
        double racc[4] = {0.0, 0.0, 0.0, 0.0};  // TT, TS, ST, SS
        // adjoint: sum_i vn_i V dq_i/dT and V dq_i/dS (the T and V/P columns
        // of J^T v from the species rows), and sum_i vn_i Q_Ns,i (the bath
        // gas's partial, which the dense rows take out of every species column)
        double aacc[3] = {0.0, 0.0, 0.0};
        // A wave's lanes take a block of 64/S consecutive reactions (inside
        // one 64-reaction chunk).  The sparse and dense Jacobian kernels'
        // waves take the blocks from a counter in LDS, the last-sorted ones
        // (falloff and third-body reactions, the costliest) first, so that a
        // wave given costly blocks takes fewer of them and all waves reach
        // the end of the loop together.  The source-term and adjoint kernels
        // keep the fixed round-robin order (the counter's code took the
        // source kernels across their 3-wave register step, and the adjoint
        // ran slower with it).
        // Deterministic accumulation: every thread runs the same number of
        // iterations over fixed blocks (lanes past the last reaction redo it
        // and add nothing); each iteration computes in parallel, then the
        // waves add their contributions one after the other.
        constexpr bool QUEUE = JAC && !DET && !ADJ;
        const int rb_lg = 6 - LG;    // log2 of the reactions per block
        const int nblk = (dm.nr + (1 << rb_lg) - 1) >> rb_lg;
        // the counter value of the wave's next block, taken during the block
        // before it (after its rates, before its LDS additions, so that the
        // return is not waited for behind them)
        int cnx = 0;
        if (QUEUE && (tid & 63) == 0) cnx = atomicAdd(bctr, 1);
        for (int pb = 0;; pb += G) {
            bool act;
            int p;
            if constexpr (!QUEUE) {
                if (DET ? pb >= dm.nr : g + pb >= dm.nr) break;
                act = !DET || g + pb < dm.nr;
                p = DET && !act ? dm.nr - 1 : g + pb;
            } else {
                const int c = __builtin_amdgcn_readfirstlane(cnx);
                if (c >= nblk) break;
                p = ((nblk - 1 - c) << rb_lg) + ((tid & 63) >> LG);
                // lanes past the last reaction redo it and add nothing (no
                // divergent continue: the wave must reach the counter together)
                act = p < dm.nr;
                if (!act) p = dm.nr - 1;
            }
            const RxnRec rr = load_rec(dm.rec + p);
            // slot positions any reaction of this 64-reaction chunk uses
            // (uniform over the wave: a wave's lanes take 64/S consecutive
            // reactions inside one chunk)
            const uint32_t cmask = __builtin_amdgcn_readfirstlane(rr.chunk);
            const bool any_rev = (cmask >> 6) & 1;
            const uint32_t w = rr.info;
            const int kind = info_kind(w);
            const bool rev = (w & INFO_REV) != 0;
            int spc[NSLOT], nu[NSLOT];
#pragma unroll
            for (int a = 0; a < NSLOT; ++a) {
                spc[a] = rr.sp[a];
                nu[a] = info_nu(w, a);
            }
            double lnA = rr.lnA, bexp = rr.b, th = rr.theta;
            if (PAR) {
                // this call's parameters (description order) instead of the
                // tables; a kernel mode of its own, so that the default kernels
                // carry none of it (their register count sits at an occupancy
                // step)
                const int o = dm.orig[p];
                lnA = dm.arr[o];
                bexp = dm.arr[dm.nr + o];
                th = dm.arr[2 * dm.nr + o];
            }
            double lnkf = lnA + bexp * lnT - th * invT;
            // a rate constant tabulated in pressure: the main expression is a factor on it
            double dlkt_dT = 0.0, dlkt_dP = 0.0;
            if (EXT && (cmask & CHUNK_TAB) && kind_table(kind)) lnkf += table_lnk(dm, kind, rr.tab, T, invT, lnT, P, dlkt_dT, dlkt_dP);
            double dG = 0.0, dH = 0.0;
            double cf[NSLOT], fr[NSLOT], dfr[NSLOT], sg[NSLOT];
#pragma unroll
            for (int a = 0; a < NSLOT; ++a) {
                sg[a] = a < MAXSIDE ? -(double)nu[a] : (double)nu[a];
                if ((cmask >> a) & 1) {
                    dG += sg[a] * AT(Gg, spc[a]);
                    dH += sg[a] * AT(H, spc[a]);
                    cf[a] = AT(C, spc[a]);
                } else {
                    cf[a] = 1.0;
                }
                powd(cf[a], nu[a], fr[a], dfr[a]);
            }
            const double dnu = rr.dnu;
            const double kf = exp(lnkf);
            const double Pf = fr[0] * fr[1] * fr[2];
            const double Pb = fr[3] * fr[4] * fr[5];
            const double lnkr = lnkf + dG - dnu * lnP0RT;
            const double kr = rev ? exp(lnkr) : 0.0;
            const double Rf = kf * Pf;
            const double Rr = kr * Pb;
            const double R = Rf - Rr;

            // third bodies with efficiency != 1, held in registers for the
            // whole iteration; the count is the chunk's largest (uniform over
            // the wave), unused entries have efficiency - 1 = 0
            const int neffc = (cmask >> 8) & 0xF;
            const int neff = (int)rr.neff;
            double Meff = 0.0;   // sum_k (alpha_k - 1) [C]_k
            if (neffc) {
                uint32_t esp[MAXEFF / 2];
                double am1[MAXEFF];
                load_eff(dm.effrec + rr.eff, neffc, esp, am1);
#pragma unroll
                for (int e = 0; e < MAXEFF; ++e)
                    if (e < neffc) Meff += am1[e] * AT(C, eff_species(esp, e));
            }

            // pressure modification
            double c = 1.0, dcdM = 0.0, dcdT = 0.0;
            // dq/d ln A = q qA - R Pr_dcdPr (adjoint): falloff Pr dc/dPr at fixed [M];
            // a chemically activated rate depends on k_inf only through Pr
            double Pr_dcdPr = 0.0, qA = 1.0;
            if (kind == K_THREEBODY || kind_falloff(kind)) {
                const double M = Ctot + Meff;
                if (kind == K_THREEBODY) {
                    c = M;
                    dcdM = 1.0;
                } else {
                    const FallRec fr_ = load_rec(dm.fall + p);
                    const double lnk0 = fr_.lnA0 + fr_.b0 * lnT - fr_.theta0 * invT;
                    const double rk = exp(lnk0 - lnkf);     // k0 / k_inf
                    const double Pr = M * rk;
                    double F = 1.0, dlF_dlP = 0.0, dlF_dT = 0.0;
                    if (kind == K_TROE) {
                        const double al = fr_.p[0], i3 = fr_.p[1], i1 = fr_.p[2], t2 = fr_.p[3];
                        const double e3 = exp(-T * i3), e1x = exp(-T * i1), e2 = exp(-t2 * invT);
                        const double Fc = (1.0 - al) * e3 + al * e1x + e2;
                        const double L = log10(Fc);
                        const double cc = -0.4 - 0.67 * L;
                        const double nn = 0.75 - 1.27 * L;
                        const double A = log10(Pr) + cc;
                        const double Bd = nn - 0.14 * A;
                        const double f = A / Bd;
                        const double den = 1.0 + f * f;
                        const double lF = L / den;
                        F = exp(LN10 * lF);
                        if (JAC) {
                            const double gg = -2.0 * L * f / (den * den);
                            dlF_dlP = gg * nn / (Bd * Bd);
                            const double df_dL = (-0.67 * Bd + 1.1762 * A) / (Bd * Bd);
                            const double dlF_dL = 1.0 / den + gg * df_dL;
                            const double dFc = -(1.0 - al) * i3 * e3 - al * i1 * e1x + t2 * invT * invT * e2;
                            dlF_dT = dlF_dL * dFc / (Fc * LN10);
                        }
                    } else if (EXT && (cmask & CHUNK_SRI) && kind == K_SRI) {
                        // F = d (a exp(-b/T) + exp(-T/c))^X T^e, X = 1 / (1 + log10(Pr)^2)
                        const double a = fr_.p[0], bb = fr_.p[1], ic = fr_.p[2], ee = fr_.p[4];
                        const double lP = log10(Pr);
                        const double X = 1.0 / (1.0 + lP * lP);
                        const double eb = exp(-bb * invT), ec = exp(-T * ic);
                        const double base = a * eb + ec;
                        const double lb = log10(base);
                        const double lF = fr_.p[3] + X * lb + ee * lnT * (1.0 / LN10);
                        F = exp(LN10 * lF);
                        if (JAC) {
                            dlF_dlP = -2.0 * lb * lP * X * X;
                            const double dbase = a * bb * invT * invT * eb - ic * ec;
                            dlF_dT = (X * dbase / base + ee * invT) * (1.0 / LN10);
                        }
                    }
                    const double ip = 1.0 / (1.0 + Pr);
                    // chemically activated: c = F / (1 + Pr) on the rate with k0,
                    // written on the rate with k_inf as F (k0 / k_inf) / (1 + Pr)
                    const bool chemact = EXT && (cmask & CHUNK_CHEMACT) && (w & INFO_CHEMACT);
                    c = chemact ? F * rk * ip : F * Pr * ip;
                    if (JAC) {
                        const double dlnPr = (fr_.b0 + fr_.theta0 * invT) * invT - (bexp + th * invT) * invT;
                        if (!chemact) {
                            const double dc_dPr = F * ip * ip + F * ip * dlF_dlP;
                            dcdM = dc_dPr * rk;
                            Pr_dcdPr = Pr * dc_dPr;
                            dcdT = dc_dPr * Pr * dlnPr + c * LN10 * dlF_dT;
                        } else {
                            // d ln c/d ln Pr = 1/(1+Pr) + d log10 F/d log10 Pr at fixed
                            // [M]; at fixed T, d ln c/d ln [M] = d log10 F/d log10 Pr -
                            // Pr/(1+Pr), and d ln q/d ln k_inf = Pr/(1+Pr) - d log10 F/d
                            // log10 Pr (both written without the cancelling 1 - 1/(1+Pr))
                            dcdM = c * (dlF_dlP / M - rk * ip);
                            dcdT = c * (ip + dlF_dlP) * dlnPr + c * LN10 * dlF_dT;
                            qA = Pr * ip - dlF_dlP;
                        }
                    }
                }
            }
            const double q = c * R;
            // production rates (the source-term kernels let an empty slot add
            // 0 to the sentinel entry, never read, instead of branching; the
            // Jacobian kernels keep the branch: without it and the T and V/P
            // rows' one they ran 2 % slower)
            auto scatter_w = [&]() {
#pragma unroll
                for (int a = 0; a < NSLOT; ++a) {
                    if (!((cmask >> a) & 1)) continue;
                    if (!JAC || nu[a]) atomicAdd(&AT(W, spc[a]), sg[a] * q);
                }
            };
            if (QUEUE && (tid & 63) == 0) cnx = atomicAdd(bctr, 1);
            if constexpr (!DET) {
                if (act) scatter_w();
            }
            // Jacobian sub-products of this reaction (what its scatter adds)
            double Qs[NSLOT], QM = 0.0, dE = 0.0, dOm = 0.0, Vt = 0.0, Vs = 0.0, bam1 = 0.0, vn = 0.0;
            if constexpr (JAC) {
            // concentration partials of q (zero for empty slots and for the
            // products of an irreversible reaction)
            const double dlnkf = (bexp + th * invT) * invT + dlkt_dT;
            const double dlnkr = dlnkf - (dH - dnu) * invT;
            const double ckf = c * kf, ckr = -c * kr;
            Qs[0] = ckf * dfr[0] * (fr[1] * fr[2]);
            Qs[1] = ckf * dfr[1] * (fr[0] * fr[2]);
            Qs[2] = ckf * dfr[2] * (fr[0] * fr[1]);
            Qs[3] = ckr * dfr[3] * (fr[4] * fr[5]);
            Qs[4] = ckr * dfr[4] * (fr[3] * fr[5]);
            Qs[5] = ckr * dfr[5] * (fr[3] * fr[4]);
            QM = R * dcdM;
            const double qT = c * (Rf * dlnkf - Rr * dlnkr) + R * dcdT;
            double Qb = 0.0, sQC = 0.0;
#pragma unroll
            for (int a = 0; a < NSLOT; ++a) sQC += Qs[a] * cf[a];
            sQC += QM * Meff;
            bam1 = rr.bam1;
            if (w & INFO_BATH) {
                // rates that depend on the bath gas: its partial Q_Ns, taken
                // out of the sum over the other species
#pragma unroll
                for (int a = 0; a < NSLOT; ++a)
                    if (spc[a] == bath) Qb += Qs[a];
                Qb += QM * bam1;
                sQC -= Qb * AT(C, bath);
            }
            const double dqdT = qT - Ctot * invT * (Qb + QM);
            const double dqdS = FORM == PJ_CONP ? -(sQC - Qb * (nsum * invV)) * invV
                                                : (Qb + QM) * invRT + q * dlkt_dP;
            dE = FORM == PJ_CONP ? dH : dH - dnu;
            dOm = rr.domega;
            if (act) {
                racc[0] += dE * dqdT;
                racc[1] += dE * dqdS;
                racc[2] += dOm * dqdT;
                racc[3] += dOm * dqdS;
            }

            // adjoint: vn = sum over the reaction's species rows of nu v, so
            // that its part of v^T J is vn times the gradient of its rate
            if constexpr (ADJ) {
#pragma unroll
                for (int a = 0; a < NSLOT; ++a) {
                    if (!((cmask >> a) & 1)) continue;
                    const bool row = nu[a] && spc[a] != bath;
                    const double vk = AT(VV, row ? 2 + spc[a] : 0);
                    vn += row ? sg[a] * vk : 0.0;
                }
            }
            if (ADJ && grad) {
                // lambda_i = v . df/dq_i, times dq_i/d ln A; summed over the
                // workgroup's states (the S lanes of this reaction are adjacent)
                const double dTdq = -T * dE / Dp;
                const double dSdq = FORM == PJ_CONP ? V * invT * dTdq + V * RU * T / P * dOm
                                                    : P * invT * dTdq + RU * T * dOm;
                const double lam = vT * dTdq + vS * dSdq + V * vn;
                // each state's own ln T and 1/T, before the sum over states
                double g0 = valid && act ? lam * (q * qA - R * Pr_dcdPr) : 0.0;
                double g1 = g0 * lnT, g2 = -g0 * invT;
                auto fold = [&](int o) {
                    g0 += __shfl_xor(g0, o, 64);
                    g1 += __shfl_xor(g1, o, 64);
                    g2 += __shfl_xor(g2, o, 64);
                };
                if constexpr (S > 0) {
#pragma unroll
                    for (int o = 1; o < S; o <<= 1) fold(o);
                } else {
                    for (int o = 1; o < SR; o <<= 1) fold(o);
                }
                if (s == 0 && act) {
                    if (gr_lds) {
                        GR[p] += g0;
                        GR[dm.nr_pad + p] += g1;
                        GR[2 * dm.nr_pad + p] += g2;
                    } else {
                        const int o = dm.orig[p];
                        atomicAdd(&grad[o], g0);
                        atomicAdd(&grad[dm.nr + o], g1);
                        atomicAdd(&grad[2 * dm.nr + o], g2);
                    }
                }
            }

            Vt = V * dqdT;
            Vs = V * dqdS;
            if (ADJ && act) {
                aacc[0] += vn * Vt;
                aacc[1] += vn * Vs;
                if ((w & INFO_BATH) && !dm.approx) aacc[2] += vn * Qb;
            }
            }

            // the Jacobian's LDS additions of this reaction
            auto scatter_j = [&]() {
            if constexpr (JAC) {
            // energy / mole weighted partials (T and V/P rows)
#pragma unroll
            for (int b = 0; b < NSLOT; ++b) {
                if (!((cmask >> b) & 1) || (b >= MAXSIDE && !any_rev)) continue;
                if (nu[b] && (b < MAXSIDE || rev)) {
                    atomicAdd(&AT(TQ, spc[b]), dE * Qs[b]);
                    atomicAdd(&AT(SQ, spc[b]), dOm * Qs[b]);
                }
            }
            // third-body partials Q_k = Q_M (alpha_k - 1), record read again
            // (cache hit) rather than held in registers across the iteration
            uint32_t esp[MAXEFF / 2];
            double qe[MAXEFF];
            if (neffc) {
                load_eff(dm.effrec + rr.eff, neffc, esp, qe);
#pragma unroll
                for (int e = 0; e < MAXEFF; ++e) {
                    qe[e] *= QM;
                    if (e < neffc && e < neff) {
                        atomicAdd(&AT(TQ, eff_species(esp, e)), dE * qe[e]);
                        atomicAdd(&AT(SQ, eff_species(esp, e)), dOm * qe[e]);
                    }
                }
            }
            if constexpr (ADJ) {
            // J^T v: the reaction adds vn Q_b to column b (the bath gas's and
            // empty slots' go to entries N and N + 1, never read; irreversible
            // products have Q_b = +-0), vn Q_k (alpha_k - 1) to third body k
#pragma unroll
            for (int b = 0; b < NSLOT; ++b) {
                if (!((cmask >> b) & 1) || (b >= MAXSIDE && !any_rev)) continue;
                atomicAdd(&AT(JTV, 2 + spc[b]), vn * Qs[b]);
            }
            if (neffc) {
#pragma unroll
                for (int e = 0; e < MAXEFF; ++e)
                    if (e < neffc) atomicAdd(&AT(JTV, 2 + eff_species(esp, e)), vn * qe[e]);
            }
            } else {
            // species rows; the slot table holds NOSLOT for pairs that do not
            // exist (empty slots, irreversible products, bath-gas columns):
            // their additions go to this lane's sink entry
            const JacRec jr = load_rec(dm.jrec + p);
            const int sink = nj + ((tid & 63) >> LG);
#pragma unroll
            for (int a = 0; a < NSLOT; ++a) {
                if (!((cmask >> a) & 1)) continue;
                const uint16_t rb = jr.rowbase[a];
                if (rb == NOSLOT) continue;
                atomicAdd(&AT(J, rb), sg[a] * Vt);
                atomicAdd(&AT(J, rb + 1), sg[a] * Vs);
#pragma unroll
                for (int b = 0; b < NSLOT; ++b) {
                    if (!((cmask >> b) & 1) || (b >= MAXSIDE && !any_rev)) continue;
                    uint16_t sl = jr.slot[a * NSLOT + b];
                    if (LS)
                        sl = nu[b] && (b < MAXSIDE || rev) && spc[b] != bath
                                 ? csr_lookup(dm, 2 + spc[a], 2 + spc[b]) : NOSLOT;
                    atomicAdd(&AT(J, sl == NOSLOT ? sink : (int)sl), sg[a] * Qs[b]);
                }
                if (neffc) {
                    // third-body columns of this row: one 16-byte load
                    const uint4 u = reinterpret_cast<const uint4*>((dm.effrec + rr.eff)->slot[a])[0];
                    const uint32_t sw[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int e = 0; e < MAXEFF; ++e) {
                        if (e >= neffc) break;
                        uint32_t sl = (sw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                        if (LS) {
                            const int sp = eff_species(esp, e);
                            sl = sp < bath ? csr_lookup(dm, 2 + spc[a], 2 + sp) : NOSLOT;
                        }
                        atomicAdd(&AT(J, sl == NOSLOT ? sink : (int)sl), sg[a] * qe[e]);
                    }
                }
            }
            if ((w & INFO_BATH) && !dm.approx) {
                // bath-gas columns of these rows go to the per-row sum B
#pragma unroll
                for (int a = 0; a < NSLOT; ++a) {
                    if (jr.rowbase[a] == NOSLOT) continue;
#pragma unroll
                    for (int b = 0; b < NSLOT; ++b)
                        if (spc[b] == bath && nu[b] && (b < MAXSIDE || rev))
                            atomicAdd(&AT(B, spc[a]), sg[a] * Qs[b]);
                    if (bam1 != 0.0) atomicAdd(&AT(B, spc[a]), sg[a] * QM * bam1);
                }
            }
            }
            }
            };
            if constexpr (!DET) {
                if (act) scatter_j();
            } else {
                for (int ow = 0; ow < nwave; ++ow) {
                    // the previous turn's LDS additions must be complete before
                    // the barrier lets the next wave add: an explicit wait (the
                    // barrier's own fence wait is not kept on this loop's back
                    // edge, and the order of the turns then slips now and then)
                    __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
                    __syncthreads();
                    if (wave == ow && act) {
                        scatter_w();
                        scatter_j();
                    }
                }
            }
        }
        __syncthreads();

        // ---- source terms (Sec. 2.2)
        // fsum: N' = sum e_k/(RT) wdot_k, Omega, then (Jacobian) sum chat_k/R
        // wdot_k and the T and V/P rows' sums, then (adjoint) the T and V/P
        // columns of J^T v from the species rows and the bath partial sum
        constexpr int NF = ADJ ? 10 : 7;
        double fsum[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) fsum[q] = 0.0;
        if (JAC) {
#pragma unroll
            for (int q = 0; q < 4; ++q) fsum[3 + q] = racc[q];
        }
        if constexpr (ADJ) {
#pragma unroll
            for (int q = 0; q < 3; ++q) fsum[7 + q] = aacc[q];
        }
        for (int k = g; k < ns; k += G) {
            const double wk = AT(W, k);
            const double ek = FORM == PJ_CONP ? AT(H, k) : AT(H, k) - 1.0;
            fsum[0] += ek * wk;
            fsum[1] += dm.wfac[k] * wk;
            if (JAC) fsum[2] += AT(CP, k) * wk;
            // CONP: d(V wdot_k)/dV = wdot_k + V dwdot_k/dV, row k's V column
            if (ADJ && FORM == PJ_CONP && k < ns - 1) fsum[8] += AT(VV, 2 + k) * wk;
        }
        block_sum<S>(fsum, red, wave, nwave, s, SR);
        const double Np = fsum[0], Om = fsum[1];
        const double Tdot = -T * Np / Dp;
        const double Sdot = FORM == PJ_CONP ? V * Tdot * invT + V * RU * T * Om / P
                                            : P * Tdot * invT + RU * T * Om;
        if (dstate && valid) {
            for (int i = g; i < N; i += G) {
                const double v = i == 0 ? Tdot : i == 1 ? Sdot : V * AT(W, i - 2);
                if (LAYOUT == PJ_LAYOUT_F) dstate[(long)i * n + st] = v;
                else dstate[st * (long)N + i] = v;
            }
        }
        if (!JAC) {
            __syncthreads();
            return;
        }

        // ---- Jacobian: T and V/P rows, closure of the species rows
        {
            const double Scw = fsum[2], TT = fsum[3], TS = fsum[4], ST = fsum[5], SS = fsum[6];
            const double cpb = AT(CP, bath);
            const double Csum = nsum * invV;
            const double dDdT = dDpdT - cpb * Ctot * invT;
            const double dDdS = FORM == PJ_CONP ? -((Dp - cpb * AT(C, bath)) - cpb * Csum) * invV
                                                : cpb / (RU * T);
            const double J00 = -(T * TT + Scw + Tdot * dDdT) / Dp;
            const double J01 = -(T * TS + Tdot * dDdS) / Dp;
            const double RTP = RU * T / P;
            // species columns: d/dn_j through [C]_j and, unless the
            // approximate form holds it fixed, the bath gas's [C]_Ns
            const double tqb = dm.approx ? 0.0 : AT(TQ, bath), sqb = dm.approx ? 0.0 : AT(SQ, bath);
            const double cpb_n = dm.approx ? 0.0 : cpb;
            for (int j = g; j < N && valid; j += G) {
                double j0, j1;
                if (j == 0) {
                    j0 = J00;
                    j1 = FORM == PJ_CONP
                             ? V * invT * J00 - V * Tdot * invT * invT + V * (RU / P) * Om + V * RTP * ST
                             : P * invT * J00 - P * Tdot * invT * invT + RU * Om + RU * T * ST;
                } else if (j == 1) {
                    j0 = J01;
                    j1 = FORM == PJ_CONP ? Tdot * invT + V * invT * J01 + RTP * Om + V * RTP * SS
                                         : Tdot * invT + P * invT * J01 + RU * T * SS;
                } else {
                    const int k = j - 2;
                    j0 = -(T * (AT(TQ, k) - tqb) + Tdot * (AT(CP, k) - cpb_n)) * invV / Dp;
                    j1 = FORM == PJ_CONP ? V * invT * j0 + RTP * (AT(SQ, k) - sqb)
                                         : P * invT * j0 + RU * T * (AT(SQ, k) - sqb) * invV;
                }
                if constexpr (ADJ) {
                    // the T and V/P rows' part, the species rows' part in the T
                    // and V/P columns, and the dense rows' bath partial (every
                    // species column)
                    AT(JTV, j) += vT * j0 + vS * j1 + (j == 0 ? fsum[7] : j == 1 ? fsum[8] : -fsum[9]);
                } else {
                    // staged in the g and h arrays (no longer needed) and
                    // written with the species rows, in output order
                    AT(Gg, j) = j0;
                    AT(H, j) = j1;
                }
            }
            if constexpr (!ADJ) {
                // bath-gas dependent rows are dense: subtract their bath partial
                for (int d = 0; d < dm.n_dense_rows; ++d) {
                    const int k = dm.dense_rows[d];
                    const int r0 = dm.row_ptr[2 + k] + 2, r1 = dm.row_ptr[3 + k];
                    const double bk = AT(B, k);
                    for (int e = r0 + g; e < r1; e += G) AT(J, e) -= bk;
                }
                if (FORM == PJ_CONP) {
                    // d(V wdot_k)/dV = wdot_k + V dwdot_k/dV
                    for (int k = g; k < ns - 1; k += G) AT(J, dm.row_ptr[2 + k] + 1) += AT(W, k);
                }
            }
        }
        __syncthreads();

        if (ADJ) {
            if (valid)
                for (int i = g; i < N; i += G) {
                    if (LAYOUT == PJ_LAYOUT_F) jac[(long)i * n + st] = AT(JTV, i);
                    else jac[st * (long)N + i] = AT(JTV, i);
                }
        } else if (SPARSE) {
            // CSR slot e of state s: the T row (e < N) and V/P row (N <= e < 2N)
            // from their staging, the species rows from the accumulator
            auto val = [&](int e, int ss) -> double {
                return e < N ? Gg[((size_t)e << LG) + ss]
                             : e < 2 * N ? H[((size_t)(e - N) << LG) + ss] : J[((size_t)e << LG) + ss];
            };
            if (LAYOUT == PJ_LAYOUT_F) {
                // S consecutive states of one slot are contiguous
                if (valid) {
                    if (dm.ccs_pos) {
                        // several column-order positions in flight per lane
                        int e = g;
                        for (; e + 7 * G < nnz; e += 8 * G) {
                            uint16_t q[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) q[u] = dm.ccs_pos[e + u * G];
#pragma unroll
                            for (int u = 0; u < 8; ++u) jac[(long)q[u] * n + st] = val(e + u * G, s);
                        }
                        for (; e < nnz; e += G) jac[(long)dm.ccs_pos[e] * n + st] = val(e, s);
                    } else
                        for (int e = g; e < nnz; e += G) jac[(long)e * n + st] = val(e, s);
                }
            } else {
                // one state's slots are contiguous: threads of one state take
                // consecutive slots
                const int s2 = tid / G, g2 = tid % G;
                const long st2 = qg * SR + s2;
                if (st2 < n) {
                    if (dm.ccs_pos) {
                        int e = g2;
                        for (; e + 7 * G < nnz; e += 8 * G) {
                            uint16_t q[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) q[u] = dm.ccs_pos[e + u * G];
#pragma unroll
                            for (int u = 0; u < 8; ++u) jac[st2 * (long)nnz + q[u]] = val(e + u * G, s2);
                        }
                        for (; e < nnz; e += G) jac[st2 * (long)nnz + dm.ccs_pos[e]] = val(e, s2);
                    } else
                        for (int e = g2; e < nnz; e += G) jac[st2 * (long)nnz + e] = val(e, s2);
                }
            }
        } else {
            // dense: every entry in output order; the species rows from the
            // accumulator through the (row, column) -> CSR slot maps (0 off
            // the pattern), the T and V/P rows from their staging
            // Each lane keeps DU map entries in flight: the map reads come from
            // L2, and one at a time they would leave the loop latency-bound
            // (16 pays where a lane has many entries, 8 where it has few; the
            // autotuner chooses)
            constexpr int DU = MODE == MODE_DENSE_U16 ? 16 : 8;
            const long NN = (long)N * N;
            if (LAYOUT == PJ_LAYOUT_F) {
                if (valid) {
                    for (int j = g; j < N; j += G) {
                        jac[st + n * ((long)N * j)] = AT(Gg, j);
                        jac[st + n * (1 + (long)N * j)] = AT(H, j);
                    }
                    long f = g;
                    for (; f + (DU - 1) * G < NN; f += DU * G) {
                        uint16_t e[DU];
#pragma unroll
                        for (int u = 0; u < DU; ++u) e[u] = dm.dmap_cm[f + u * G];
#pragma unroll
                        for (int u = 0; u < DU; ++u)
                            if (e[u] != DMAP_SKIP) jac[st + n * (f + u * G)] = e[u] == NOSLOT ? 0.0 : AT(J, e[u]);
                    }
                    for (; f < NN; f += G) {
                        const uint16_t e = dm.dmap_cm[f];
                        if (e == DMAP_SKIP) continue;
                        jac[st + n * f] = e == NOSLOT ? 0.0 : AT(J, e);
                    }
                }
            } else {
                const int s2 = tid / G, g2 = tid % G;
                const long st2 = qg * SR + s2;
                if (st2 < n) {
                    double* out = jac + st2 * NN;
                    for (int f = g2; f < 2 * N; f += G)
                        out[f] = f < N ? Gg[((size_t)f << LG) + s2] : H[((size_t)(f - N) << LG) + s2];
                    long f = 2 * N + g2;
                    for (; f + (DU - 1) * G < NN; f += DU * G) {
                        uint16_t e[DU];
#pragma unroll
                        for (int u = 0; u < DU; ++u) e[u] = dm.dmap_rm[f + u * G];
#pragma unroll
                        for (int u = 0; u < DU; ++u)
                            out[f + u * G] = e[u] == NOSLOT ? 0.0 : J[((size_t)e[u] << LG) + s2];
                    }
                    for (; f < NN; f += G) {
                        const uint16_t e = dm.dmap_rm[f];
                        out[f] = e == NOSLOT ? 0.0 : J[((size_t)e << LG) + s2];
                    }
                }
            }
        }
        __syncthreads();
        }
#undef AT
}

// LDS offset (doubles) of the adjoint's per-workgroup parameter sums
__device__ inline size_t gr_offset(const DevMech& dm, int S, int nwave) {
    return ((size_t)5 * (dm.ns + 1) + (size_t)RED_PER_WAVE * nwave + 2 * (size_t)dm.N + dm.ns +
            2 * (size_t)dm.N + 2) * S;
}

// Groups of S consecutive states.  Consecutive groups go to workgroups of
// the same XCD (workgroups are handed to the 8 XCDs round-robin), so that the
// partial cache lines of layout-F arrays of neighbouring states meet in one
// L2: XCD x takes the contiguous range [ng x/8, ng (x+1)/8).
__device__ inline void group_range(long ngroups, long& q0, long& q1, long& qstep) {
    q0 = blockIdx.x;
    q1 = ngroups;
    qstep = gridDim.x;
    if (gridDim.x >= 8 && (gridDim.x & 7) == 0) {
        const long x = blockIdx.x & 7;
        q0 = ngroups * x / 8 + (blockIdx.x >> 3);
        q1 = ngroups * (x + 1) / 8;
        qstep = gridDim.x >> 3;
    }
}

// (source terms: held to the register count of 3 waves per SIMD; the
// compiler otherwise gives some state counts a few registers more and two
// waves per SIMD)
template <int FORM, int LAYOUT, int MODE, int S, bool EXT>
__global__ void __launch_bounds__(MAX_THREADS) __attribute__((amdgpu_waves_per_eu(base_mode(MODE) == MODE_SRC ? 3 : 1)))
pj_kernel(const DevMech dm, const long n,
                                                          const double* __restrict__ state,
                                                          const double* __restrict__ param,
                                                          double* __restrict__ dstate,
                                                          double* __restrict__ jac,
                                                          const double* __restrict__ vin,
                                                          double* __restrict__ grad,
                                                          const int grad_in_lds) {
    extern __shared__ double lds[];
    constexpr bool ADJ = base_mode(MODE) == MODE_ADJ;
    const int tid = threadIdx.x, nthr = blockDim.x;
    double* GR = lds + gr_offset(dm, S, nthr >> 6);
    long q0, q1, qstep;
    group_range((n + S - 1) / S, q0, q1, qstep);
    // adjoint parameter sums: in LDS per workgroup when they fit (added to
    // the output once at the end), else added to the output per group
    const bool gr_lds = ADJ && grad && grad_in_lds;
    if (gr_lds) {
        for (int i = tid; i < 3 * dm.nr_pad; i += nthr) GR[i] = 0.0;
        __syncthreads();
    }
    for (long qg = q0; qg < q1; qg += qstep)
        eval_group<FORM, LAYOUT, MODE, S, EXT>(dm, n, state, param, dstate, jac, vin, grad, gr_lds, GR, qg);
    if (gr_lds) {
        // the workgroup's sums into the batch sums, in description order
        for (int i = tid; i < dm.nr; i += nthr) {
            const int o = dm.orig[i];
            atomicAdd(&grad[o], GR[i]);
            atomicAdd(&grad[dm.nr + o], GR[dm.nr_pad + i]);
            atomicAdd(&grad[2 * dm.nr + o], GR[2 * dm.nr_pad + i]);
        }
    }
}

// Ragged batch: the segments (each a mechanism with its own states and
// outputs) share one launch; the global group index runs over the segments'
// groups in order, so every workgroup of the persistent grid takes groups of
// any segment.
// Adjoint parameter sums of one segment, kept in LDS, into its output.
__device__ inline void flush_gr(const BatchSeg& b, const double* GR) {
    __syncthreads();
    if (b.grad)
        for (int i = threadIdx.x; i < b.dm.nr; i += blockDim.x) {
            const int o = b.dm.orig[i];
            atomicAdd(&b.grad[o], GR[i]);
            atomicAdd(&b.grad[b.dm.nr + o], GR[b.dm.nr_pad + i]);
            atomicAdd(&b.grad[2 * b.dm.nr + o], GR[2 * b.dm.nr_pad + i]);
        }
    __syncthreads();
}

// (source terms: held to the register count of 3 waves per SIMD, as the
// per-mechanism source kernel is).  SU > 0: every segment takes SU states
// per group, a compile-time body; SU = 0: each its own, read at run time.
template <int FORM, int LAYOUT, int MODE, bool EXT, int SU>
__global__ void __launch_bounds__(MAX_THREADS) __attribute__((amdgpu_waves_per_eu(MODE == MODE_SRC ? 3 : 1)))
pj_batch_kernel(const BatchSeg* __restrict__ segs, const int nseg, const long total) {
    extern __shared__ double lds[];
    // Every segment is spread over the whole grid, each XCD taking a
    // contiguous share of it as for a single mechanism, so that segments of
    // very different cost per group keep all XCDs equally busy.  Each segment
    // has its own states per group (a run-time value of the one group body).
    // Adjoint: the parameter sums of the segment in hand live in LDS at its
    // gr_off, after its states' arrays (gr_off < 0: added to the output per
    // group), and are flushed once per segment.
    for (int k = 0; k < nseg; ++k) {
        const BatchSeg& b = segs[k];
        const bool use_gr = MODE == MODE_ADJ && b.gr_off >= 0;
        double* GR = use_gr ? lds + b.gr_off : nullptr;
        const long ng = (k + 1 < nseg ? segs[k + 1].g0 : total) - b.g0;
        long q0, q1, qstep;
        group_range(ng, q0, q1, qstep);
        if (q0 >= q1) continue;   // uniform over the workgroup
        if (use_gr) {
            for (int i = threadIdx.x; i < 3 * b.dm.nr_pad; i += blockDim.x) GR[i] = 0.0;
            __syncthreads();
        }
        const int bs = SU > 0 ? SU : b.S;
        for (long q = q0; q < q1; q += qstep)
            eval_group<FORM, LAYOUT, MODE, SU, EXT>(b.dm, b.n, b.state, b.param, b.dstate, b.out, b.vin,
                                                   b.grad, use_gr && b.grad, GR, q, bs);
        if (use_gr) flush_gr(b, GR);
    }
}

// Allow a kernel the device's whole LDS per workgroup, once per device (the
// attribute belongs to the function, not to a launch).
inline hipError_t allow_full_lds(const void* fn, std::atomic<uint64_t>& done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? (1ull << dev) : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    int mx = 0;
    e = hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

template <int FORM, int LAYOUT, int MODE, int S, bool EXT>
static hipError_t launch_t(const DevMech& dm, int64_t n, const double* state, const double* param,
                           double* dstate, double* jac, const double* vin, double* grad,
                           int grad_in_lds, int waves, int64_t lds, hipStream_t stream) {
    auto k = pj_kernel<FORM, LAYOUT, MODE, S, EXT>;
    if (lds > 65536) {
        static std::atomic<uint64_t> done{0};
        hipError_t e = allow_full_lds((const void*)k, done);
        if (e != hipSuccess) return e;
    }
    // one workgroup per group of S states, rounded down to a multiple of 8
    // (the XCD count)
    const int64_t groups = (n + S - 1) / S;
    // the adjoint's workgroups each add their parameter sums to the output
    // once: a bounded, persistent grid keeps those atomics few
    constexpr bool ADJ = base_mode(MODE) == MODE_ADJ;
    const int64_t cap = ADJ ? 2048 : (1 << 30);
    int64_t grid = groups < cap ? groups : cap;
    if (grid >= 8) grid &= ~(int64_t)7;
    if (ADJ && grad) {
        hipError_t e = zero_async(grad, 3 * (int64_t)dm.nr, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * waves), (size_t)lds, stream, dm, (long)n,
                       state, param, dstate, jac, vin, grad, grad_in_lds);
    return hipGetLastError();
}

template <int FORM, int LAYOUT, int MODE, bool EXT, int SU>
static hipError_t launch_batch_t(int waves, int64_t lds, const BatchSeg* segs, int nseg, int64_t total,
                                 hipStream_t stream) {
    auto k = pj_batch_kernel<FORM, LAYOUT, MODE, EXT, SU>;
    if (lds > 65536) {
        static std::atomic<uint64_t> done{0};
        hipError_t e = allow_full_lds((const void*)k, done);
        if (e != hipSuccess) return e;
    }
    // a persistent grid over the segments' groups (a multiple of 8, the XCD count)
    // (the adjoint's workgroups each flush their parameter sums once per
    // segment: a smaller grid keeps those atomics few)
    const int64_t cap = MODE == MODE_ADJ ? 2048 : 8192;
    int64_t grid = total < cap ? total : cap;
    if (grid >= 8) grid &= ~(int64_t)7;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * waves), (size_t)lds, stream, segs, nseg, (long)total);
    return hipGetLastError();
}


// Launch of one instantiation set of one form: EXT = false for mechanisms of
// elementary, third-body, Lindemann and Troe reactions only (none of the
// further types' code is compiled in), EXT = true otherwise.  The four sets
// (EXT x form) are instantiated in four translation units, which build in
// parallel.
template <bool EXT, int FORM>
hipError_t launch_impl(const DevMech& dm, int mode, int form, int layout, int S, int64_t n,
                       const double* state, const double* param, double* dstate, double* jac,
                       const double* vin, double* grad, int grad_in_lds, int waves, int64_t lds,
                       hipStream_t stream) {
#define PJ_CASE(F, L, M, SS)                                                                 \
    if (form == F && layout == L && mode == M && S == SS)                                    \
        return launch_t<F, L, M, SS, EXT>(dm, n, state, param, dstate, jac, vin, grad, grad_in_lds, \
                                          waves, lds, stream);
#define PJ_S(F, L, M)                                                                        \
    PJ_CASE(F, L, M, 1) PJ_CASE(F, L, M, 2) PJ_CASE(F, L, M, 4) PJ_CASE(F, L, M, 8)          \
    PJ_CASE(F, L, M, 16) PJ_CASE(F, L, M, 32) PJ_CASE(F, L, M, 64)
#define PJ_SA(F, L) PJ_CASE(F, L, MODE_ADJ, 1) PJ_CASE(F, L, MODE_ADJ, 2) PJ_CASE(F, L, MODE_ADJ, 4)
#define PJ_SL(F, L) PJ_CASE(F, L, MODE_SPARSE_LS, 1) PJ_CASE(F, L, MODE_SPARSE_LS, 2) PJ_CASE(F, L, MODE_SPARSE_LS, 4)
#define PJ_SAP(F, L) PJ_CASE(F, L, MODE_ADJ_P, 1) PJ_CASE(F, L, MODE_ADJ_P, 2) PJ_CASE(F, L, MODE_ADJ_P, 4)
#define PJ_SU(F, L) PJ_CASE(F, L, MODE_DENSE_U16, 1) PJ_CASE(F, L, MODE_DENSE_U16, 2) PJ_CASE(F, L, MODE_DENSE_U16, 4)
#define PJ_SD(F, L) PJ_CASE(F, L, MODE_SRC_DET, 1) PJ_CASE(F, L, MODE_SRC_DET, 2) PJ_CASE(F, L, MODE_SRC_DET, 4) \
    PJ_CASE(F, L, MODE_SPARSE_DET, 1) PJ_CASE(F, L, MODE_SPARSE_DET, 2) PJ_CASE(F, L, MODE_SPARSE_DET, 4)
#define PJ_MODES(F, L) PJ_S(F, L, MODE_SRC) PJ_S(F, L, MODE_SPARSE) PJ_S(F, L, MODE_DENSE) PJ_SA(F, L) PJ_SL(F, L) \
    PJ_S(F, L, MODE_SRC_P) PJ_SAP(F, L) PJ_SD(F, L) PJ_SU(F, L)
    PJ_MODES(FORM, PJ_LAYOUT_F)
    PJ_MODES(FORM, PJ_LAYOUT_C)
#undef PJ_MODES
#undef PJ_SD
#undef PJ_SU
#undef PJ_SAP
#undef PJ_SL
#undef PJ_SA
#undef PJ_S
#undef PJ_CASE
    return hipErrorInvalidValue;
}

template <bool EXT>
hipError_t launch_batch_impl(int mode, int form, int layout, int waves, int64_t lds, const BatchSeg* d_segs,
                             int nseg, int64_t total, int su, hipStream_t stream) {
#define PJ_BCASE(F, L, M)                                                                       \
    if (form == F && layout == L && mode == M) {                                                \
        if (su == 1) return launch_batch_t<F, L, M, EXT, 1>(waves, lds, d_segs, nseg, total, stream); \
        if (su == 2) return launch_batch_t<F, L, M, EXT, 2>(waves, lds, d_segs, nseg, total, stream); \
        if (su == 4) return launch_batch_t<F, L, M, EXT, 4>(waves, lds, d_segs, nseg, total, stream); \
        return launch_batch_t<F, L, M, EXT, 0>(waves, lds, d_segs, nseg, total, stream);            \
    }
#define PJ_BMODES(F, L) PJ_BCASE(F, L, MODE_SRC) PJ_BCASE(F, L, MODE_SPARSE) PJ_BCASE(F, L, MODE_ADJ)
    PJ_BMODES(PJ_CONP, PJ_LAYOUT_F)
    PJ_BMODES(PJ_CONP, PJ_LAYOUT_C)
    PJ_BMODES(PJ_CONV, PJ_LAYOUT_F)
    PJ_BMODES(PJ_CONV, PJ_LAYOUT_C)
#undef PJ_BMODES
#undef PJ_BCASE
    return hipErrorInvalidValue;
}

}  // namespace pj
