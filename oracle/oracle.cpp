// Oracle: a plain, slow, serial FP64 CPU evaluation of the thermochemical
// source terms and the analytical chemical-kinetic Jacobian of Curtis,
// Niemeyer & Sung (pyJac v2, arXiv:1809.01029), Sec. 2.2.
//
// THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark load it.  It shares no code with the GPU
// library: it parses the mechanism description itself, evaluates everything
// with dense loops in the order the formulas are written, and uses no tables
// derived by the library.
//
// Everything is templated on the scalar type S:
//   * double                 - the values;
//   * std::complex<double>   - complex-step derivatives (a check of the
//                              hand-derived Jacobian, exact to rounding);
//   * Err                    - value plus a first-order bound on its rounding
//                              error (running error analysis: Wilkinson;
//                              Higham, Accuracy and Stability of Numerical
//                              Algorithms, Sec. 3.3).  Each operation adds the
//                              propagated bounds of its operands, weighted by
//                              the magnitude of its partial derivatives, and
//                              one rounding of its own result; library exp
//                              and log add one ulp.  Parity tolerances widen
//                              by this bound only where it is not small
//                              against the value (cancellation);
//   * long double            - the same definitions in 64-bit-significand
//                              arithmetic, an independent reference against
//                              which the bound is checked;
//   * Cnt                    - values that count the arithmetic operations
//                              of the source terms as written here (the
//                              algorithmic operation count of the roofline).
//
// The adjoint (the product of the transposed Jacobian with a vector v and
// the batch-summed derivatives of v . dPhi/dt with respect to every
// reaction's Arrhenius parameters ln A, b and Ea/R) is written from the same
// definitions: J^T v from the analytical Jacobian, and the parameter
// derivatives by the chain rule through the rate of progress (for falloff
// reactions the parameters are those of the high-pressure limit).
//
// Reaction types (Sec. 2.2 names them as supported; the formulas are the
// standard ones): elementary, third-body, falloff with the Lindemann, Troe or
// SRI broadening factor, chemically activated (the same broadening on a rate
// with the low-pressure limit, c = F / (1 + Pr)), pressure-dependent
// Arrhenius (P-Log: ln k linear in ln P between tabulated pressures, the end
// values outside) and Chebyshev (log10 k a double Chebyshev series in reduced
// 1/T and log P).  For the last two the main Arrhenius expression is a factor
// on the tabulated rate, which is what the adjoint's parameters then mean; a
// rate tabulated in pressure depends on the state variable P of the
// constant-volume form.
//
// The "approximate" Jacobian (Sec. 3.4) neglects the dependence of the bath
// gas's concentration on the other species' moles: d[C]_Ns/dn_j = 0 for
// j < Ns, while its dependence on T and V (or P) is kept; this removes the
// dense rows the bath gas would otherwise create.
//
// Units: SI with kmol.  R_u = 8314.462618 J/(kmol K), P_ref = 101325 Pa.
// State vector (Sec. 2.2): Phi = (T, V, n_1..n_{Ns-1}) for constant pressure
// (parameter P) and (T, P, n_1..n_{Ns-1}) for constant volume (parameter V);
// the last species is the bath gas, closed by the ideal-gas law.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <set>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

namespace {

const double RU = 8314.462618;
const double PREF = 101325.0;
const double LN10 = 2.302585092994045684;

enum { FORM_CONP = 0, FORM_CONV = 1 };
enum { T_ELEM = 0, T_THREEBODY = 1, T_LINDEMANN = 2, T_TROE = 3, T_SRI = 4, T_PLOG = 5, T_CHEB = 6 };

struct Species {
    double W;
    int comp[4];
    double tlow, tmid, thigh;
    double alo[7], ahi[7];
};

struct Reaction {
    int type;
    bool rev;
    std::vector<std::pair<int, int>> reac, prod;   // (species, coefficient)
    double lnA, b, theta;
    double lnA0 = 0, b0 = 0, theta0 = 0;            // low-pressure limit
    double alpha = 0, T3 = 0, T1 = 0, T2 = 0;       // Troe
    double sri[5] = {0, 0, 0, 0, 0};                // SRI a, b, c, d, e
    bool chemact = false;                           // chemically activated
    std::vector<std::pair<int, double>> eff;        // (species, efficiency)
    // P-Log: (P [Pa], ln A, b, Ea/R) in ascending pressure
    std::vector<std::vector<double>> plog;
    // Chebyshev: NT x NP coefficients of log10 k (t-major) over [Tmin, Tmax] x [Pmin, Pmax]
    int cheb_nt = 0, cheb_np = 0;
    double cheb_Tmin = 0, cheb_Tmax = 0, cheb_Pmin = 0, cheb_Pmax = 0;
    std::vector<double> cheb;
    bool falloff() const { return type == T_LINDEMANN || type == T_TROE || type == T_SRI; }
    bool pressure_table() const { return type == T_PLOG || type == T_CHEB; }
};

struct Mech {
    int ns = 0;
    std::vector<Species> sp;
    std::vector<Reaction> rx;
};

// ---------------------------------------------------------------------------
// scalar types

// Running error bound: v is the computed value, m a bound on |v - exact| in
// units of the unit roundoff u = 2^-53 (to first order in u).  Inputs and the
// constants of the description are exact (m = 0).
const double U_ROUND = 1.1102230246251565e-16;   // 2^-53
const double FN_ULPS = 2.0;   // library exp / log / log10: within one ulp (2u)

struct Err {
    double v, m;
    Err() : v(0), m(0) {}
    Err(double x) : v(x), m(0) {}
    Err(double x, double mm) : v(x), m(mm) {}
};
inline Err operator+(Err a, Err b) { double r = a.v + b.v; return Err(r, a.m + b.m + std::fabs(r)); }
inline Err operator-(Err a, Err b) { double r = a.v - b.v; return Err(r, a.m + b.m + std::fabs(r)); }
inline Err operator-(Err a) { return Err(-a.v, a.m); }
inline Err operator*(Err a, Err b) {
    double r = a.v * b.v;
    return Err(r, std::fabs(b.v) * a.m + std::fabs(a.v) * b.m + std::fabs(r));
}
// d(a/b) = da / b - (a/b) db / b
inline Err operator/(Err a, Err b) {
    double r = a.v / b.v;
    return Err(r, (a.m + std::fabs(r) * b.m) / std::fabs(b.v) + std::fabs(r));
}
inline Err& operator+=(Err& a, Err b) { a = a + b; return a; }
inline Err& operator-=(Err& a, Err b) { a = a - b; return a; }
inline Err exp(Err a) { double e = std::exp(a.v); return Err(e, e * a.m + FN_ULPS * e); }
inline Err log(Err a) {
    double l = std::log(a.v);
    return Err(l, a.m / std::fabs(a.v) + FN_ULPS * std::fabs(l));
}
inline Err log10(Err a) {
    double l = std::log10(a.v);
    return Err(l, a.m / (LN10 * std::fabs(a.v)) + FN_ULPS * std::fabs(l));
}

// Operation counting: every + - * / of two values (or a value and a
// constant) counts one, exp, log and log10 count separately.  A
// transcendental of an argument already taken in the same evaluation counts
// once (a common subexpression: ln T enters every rate constant and every
// species entropy as written here).
struct OpCount {
    double flops = 0, exps = 0, logs = 0, log10s = 0;
    std::set<std::pair<int, uint64_t>> seen;
    bool fresh(int fn, double arg) {
        uint64_t bits;
        std::memcpy(&bits, &arg, sizeof bits);
        return seen.insert({fn, bits}).second;
    }
};
thread_local OpCount g_ops;
// Set while counting the operations of the source terms alone: the
// evaluation then skips the derivatives it otherwise forms along the way
// (for the Jacobian and the parameter gradient).  Values are unchanged.
thread_local bool g_values_only = false;
struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
};
inline Cnt operator+(Cnt a, Cnt b) { g_ops.flops += 1; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { g_ops.flops += 1; return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { g_ops.flops += 1; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { g_ops.flops += 1; return Cnt(a.v / b.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt exp(Cnt a) { if (g_ops.fresh(0, a.v)) g_ops.exps += 1; return Cnt(std::exp(a.v)); }
inline Cnt log(Cnt a) { if (g_ops.fresh(1, a.v)) g_ops.logs += 1; return Cnt(std::log(a.v)); }
inline Cnt log10(Cnt a) { if (g_ops.fresh(2, a.v)) g_ops.log10s += 1; return Cnt(std::log10(a.v)); }

inline double re(double x) { return x; }
inline double re(const std::complex<double>& x) { return x.real(); }
inline double re(const Err& x) { return x.v; }
inline double re(const Cnt& x) { return x.v; }
inline double re(long double x) { return (double)x; }

using std::exp;
using std::log;
using std::log10;

// The closure needs the exactly rounded sum of the species moles
// (s = RN(sum_k n_k)), so that it does not depend on a summation order.
// Quad precision (113-bit significand) gives it except for exact ties.
inline double rn_sum(const double* v, int n) {
    __float128 acc = 0;
    for (int k = 0; k < n; ++k) acc += (__float128)v[k];
    return (double)acc;
}
inline double exact_sum(const double* v, int n) { return rn_sum(v, n); }
template <class S>
S exact_sum(const S* v, int n) {
    std::vector<double> x(n);
    for (int k = 0; k < n; ++k) x[k] = re(v[k]);
    return S(rn_sum(x.data(), n));
}
inline std::complex<double> exact_sum(const std::complex<double>* v, int n) {
    std::vector<double> x(n);
    double im = 0;
    for (int k = 0; k < n; ++k) { x[k] = v[k].real(); im += v[k].imag(); }
    return std::complex<double>(rn_sum(x.data(), n), im);
}

// ---------------------------------------------------------------------------
// description parsing

int type_code(const std::string& t) {
    if (t == "ELEM") return T_ELEM;
    if (t == "THREEBODY") return T_THREEBODY;
    if (t == "LINDEMANN") return T_LINDEMANN;
    if (t == "TROE") return T_TROE;
    if (t == "SRI") return T_SRI;
    if (t == "PLOG") return T_PLOG;
    if (t == "CHEB") return T_CHEB;
    return -1;
}

bool parse(const char* path, Mech& m) {
    std::ifstream f(path);
    if (!f) return false;
    std::string tok;
    int ver;
    if (!(f >> tok >> ver) || tok != "PJMECH" || ver != 1) return false;
    int ns;
    if (!(f >> tok >> ns) || tok != "SPECIES" || ns < 2) return false;
    m.ns = ns;
    m.sp.resize(ns);
    for (int k = 0; k < ns; ++k) {
        Species& s = m.sp[k];
        int idx;
        std::string name;
        if (!(f >> tok >> idx >> name >> s.W) || tok != "SP" || idx != k) return false;
        for (int e = 0; e < 4; ++e) f >> s.comp[e];
        f >> s.tlow >> s.tmid >> s.thigh;
        for (int c = 0; c < 7; ++c) f >> s.alo[c];
        for (int c = 0; c < 7; ++c) f >> s.ahi[c];
        if (!f) return false;
    }
    int nr;
    if (!(f >> tok >> nr) || tok != "REACTIONS" || nr < 0) return false;
    m.rx.resize(nr);
    f >> tok;
    for (int i = 0; i < nr; ++i) {
        Reaction& r = m.rx[i];
        int idx, rev, n;
        std::string typ;
        if (tok != "RX" || !(f >> idx >> typ >> rev >> n) || idx != i) return false;
        r.type = type_code(typ);
        if (r.type < 0) return false;
        r.rev = rev != 0;
        for (int a = 0; a < n; ++a) { int s, nu; f >> s >> nu; r.reac.push_back({s, nu}); }
        f >> n;
        for (int a = 0; a < n; ++a) { int s, nu; f >> s >> nu; r.prod.push_back({s, nu}); }
        f >> r.lnA >> r.b >> r.theta;
        while (f >> tok) {
            if (tok == "LOW") f >> r.lnA0 >> r.b0 >> r.theta0;
            else if (tok == "TROE") f >> r.alpha >> r.T3 >> r.T1 >> r.T2;
            else if (tok == "SRI") { for (double& v : r.sri) f >> v; }
            else if (tok == "CHEMACT") r.chemact = true;
            else if (tok == "PLOG") {
                f >> n;
                for (int a = 0; a < n; ++a) {
                    std::vector<double> pt(4);
                    for (double& v : pt) f >> v;
                    r.plog.push_back(pt);
                }
            } else if (tok == "CHEB") {
                f >> r.cheb_nt >> r.cheb_np >> r.cheb_Tmin >> r.cheb_Tmax >> r.cheb_Pmin >> r.cheb_Pmax;
                if (!f || r.cheb_nt < 1 || r.cheb_np < 1) return false;
                r.cheb.resize((size_t)r.cheb_nt * r.cheb_np);
                for (double& v : r.cheb) f >> v;
            } else if (tok == "EFF") {
                f >> n;
                for (int a = 0; a < n; ++a) { int s; double al; f >> s >> al; r.eff.push_back({s, al}); }
            } else break;
        }
        if (!f) return false;
        if ((r.type == T_PLOG) != !r.plog.empty() || (r.type == T_CHEB) != !r.cheb.empty()) return false;
        for (size_t a = 0; a < r.plog.size(); ++a)
            if (!(r.plog[a][0] > 0) || (a && !(r.plog[a][0] > r.plog[a - 1][0]))) return false;
        if (r.type == T_CHEB && !(r.cheb_Tmin > 0 && r.cheb_Tmax > r.cheb_Tmin && r.cheb_Pmin > 0
                                  && r.cheb_Pmax > r.cheb_Pmin)) return false;
        if (r.chemact && !r.falloff()) return false;
    }
    return tok == "END";
}

// ---------------------------------------------------------------------------
// species thermodynamics: NASA 7-coefficient polynomials (Sec. 2.2, the
// temperature source term uses H, U, Cp and Cv of each species)

template <class S>
struct Thermo {
    S cp;      // Cp / R
    S h;       // H / (R T)
    S s;       // S / R
    S dcp;     // d(Cp/R)/dT
    S dh;      // d(H/(R T))/dT
    S ds;      // d(S/R)/dT
};

template <class S>
Thermo<S> species_thermo(const Species& sp, S T) {
    const double* a = re(T) < sp.tmid ? sp.alo : sp.ahi;
    S T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    Thermo<S> t;
    t.cp = S(a[0]) + S(a[1]) * T + S(a[2]) * T2 + S(a[3]) * T3 + S(a[4]) * T4;
    t.h = S(a[0]) + S(a[1]) * T / S(2.0) + S(a[2]) * T2 / S(3.0) + S(a[3]) * T3 / S(4.0)
          + S(a[4]) * T4 / S(5.0) + S(a[5]) / T;
    t.s = S(a[0]) * log(T) + S(a[1]) * T + S(a[2]) * T2 / S(2.0) + S(a[3]) * T3 / S(3.0)
          + S(a[4]) * T4 / S(4.0) + S(a[6]);
    if (g_values_only) return t;
    t.dcp = S(a[1]) + S(2.0 * a[2]) * T + S(3.0 * a[3]) * T2 + S(4.0 * a[4]) * T3;
    t.dh = S(a[1]) / S(2.0) + S(2.0 * a[2]) * T / S(3.0) + S(3.0 * a[3]) * T2 / S(4.0)
           + S(4.0 * a[4]) * T3 / S(5.0) - S(a[5]) / T2;
    t.ds = S(a[0]) / T + S(a[1]) + S(a[2]) * T + S(a[3]) * T2 + S(a[4]) * T3;
    return t;
}

// ---------------------------------------------------------------------------
// the thermochemical state and its concentrations

template <class S>
struct State {
    S T, V, P;
    std::vector<S> C;     // [C]_k for all Ns species, kmol/m^3
    std::vector<S> n;     // moles of all Ns species
};

// [C]_k = n_k / V (Sec. 2.2); the bath gas from the ideal gas law P V = n R T:
// n_Ns = P V / (R T) - RN(sum_{k<Ns} n_k).
// frozen = true: the bath gas's moles do not follow the other species' moles
// (the sum's imaginary part is dropped), the complex-step form of the
// approximate Jacobian
inline std::complex<double> frozen_sum(const std::complex<double>* v, int n) {
    std::vector<double> x(n);
    for (int k = 0; k < n; ++k) x[k] = v[k].real();
    return std::complex<double>(rn_sum(x.data(), n), 0.0);
}
template <class S>
S frozen_sum(const S* v, int n) { return exact_sum(v, n); }

// The bath gas's moles are defined on the double inputs: n_Ns = PV/(RT) -
// RN(sum_k n_k), formed as (P V) / (R T) minus that sum, in double, so that
// any two codes that follow the definition hold the same bits.  The types
// that measure rounding (Err) or carry more precision (long double) take
// that double as their exact starting point; the complex step and the
// operation count follow the arithmetic as written.
template <class S>
S closure_moles(S ntot, S sum, double) { return ntot - sum; }
inline Err closure_moles(Err, Err, double shared) { return Err(shared, 0.0); }
inline long double closure_moles(long double, long double, double shared) { return (long double)shared; }

template <class S>
State<S> make_state(const Mech& m, int form, const S* x, S param, bool frozen = false) {
    State<S> st;
    int ns = m.ns;
    st.T = x[0];
    if (form == FORM_CONP) { st.V = x[1]; st.P = param; }
    else { st.P = x[1]; st.V = param; }
    S ntot = (st.P * st.V) / (S(RU) * st.T);
    S sum = frozen ? frozen_sum(x + 2, ns - 1) : exact_sum(x + 2, ns - 1);
    std::vector<double> xd(ns - 1);
    for (int k = 0; k < ns - 1; ++k) xd[k] = re(x[2 + k]);
    const double shared = (re(st.P) * re(st.V)) / (RU * re(st.T)) - rn_sum(xd.data(), ns - 1);
    st.n.resize(ns);
    st.C.resize(ns);
    for (int k = 0; k < ns - 1; ++k) st.n[k] = x[2 + k];
    st.n[ns - 1] = closure_moles(ntot, sum, shared);
    for (int k = 0; k < ns; ++k) st.C[k] = st.n[k] / st.V;
    return st;
}

// ---------------------------------------------------------------------------
// reaction rates (Sec. 2.2: wdot_k = sum_i nu_ki R_i c_i)

template <class S>
struct RxnEval {
    S kf, kr, c, Rf, Rr, q;
    // derivatives, used by the Jacobian
    S dkf_dT, dkr_dT;
    S dc_dT;                    // at fixed concentrations
    std::vector<S> dc_dC;       // dc/d[C]_m, all species, at fixed C_tot
    S dc_dCtot;                 // dc/dC_tot at fixed species concentrations
    std::vector<S> dRf_dC, dRr_dC;
    S dRf_dT, dRr_dT;
    std::vector<S> dq_dC;       // dq/d[C]_m at fixed T and C_tot
    S dq_dCtot;                 // dq/dC_tot at fixed T and concentrations
    S dq_dT;                    // dq/dT at fixed concentrations (and fixed P)
    S dq_dP;                    // dq/dP at fixed T and concentrations (P-Log, Chebyshev)
    S dq_dlnk;                  // dq/d ln(main Arrhenius factor) at fixed T and concentrations
};

// Optional perturbations of a reaction's Arrhenius parameters (ln A, b,
// Ea/R) of k_f (k_inf for falloff), used by the complex-step check of the
// parameter derivatives; nullptr everywhere else.
template <class S>
struct ParamShift {
    S lnA, b, theta;
};

template <class S>
S arrhenius(double lnA, double b, double theta, S T) {
    return exp(S(lnA) + S(b) * log(T) - S(theta) / T);
}

template <class S>
S ipow(S x, int nu) {
    S r(1.0);
    for (int a = 0; a < nu; ++a) r = r * x;
    return r;
}

// product of [C]^nu over a side of the reaction, and its derivative by [C]_m
template <class S>
S mass_action(const std::vector<std::pair<int, int>>& side, const std::vector<S>& C) {
    S p(1.0);
    for (auto& e : side) p = p * ipow(C[e.first], e.second);
    return p;
}
template <class S>
S mass_action_d(const std::vector<std::pair<int, int>>& side, const std::vector<S>& C, int m) {
    S d(0.0);
    for (size_t a = 0; a < side.size(); ++a) {
        if (side[a].first != m) continue;
        int nu = side[a].second;
        S t = S((double)nu) * ipow(C[m], nu - 1);
        for (size_t b = 0; b < side.size(); ++b)
            if (b != a) t = t * ipow(C[side[b].first], side[b].second);
        d = d + t;
    }
    return d;
}

// Rate constants tabulated in pressure: ln k and its partial derivatives by T
// (at fixed P) and by ln P (at fixed T).
template <class S>
struct LnK {
    S v, dT, dlnP;
};

// P-Log: between the two tabulated pressures that bracket P, ln k is linear in
// ln P, each pressure carrying its own Arrhenius expression; below the first
// or above the last pressure that end's expression holds.
template <class S>
LnK<S> plog_lnk(const Reaction& r, S T, S P) {
    auto lnk_at = [&](const std::vector<double>& pt, S& dT) {
        dT = S(pt[2]) / T + S(pt[3]) / (T * T);
        return S(pt[1]) + S(pt[2]) * log(T) - S(pt[3]) / T;
    };
    LnK<S> o;
    const size_t m = r.plog.size();
    const double p = re(P);
    o.dlnP = S(0.0);
    if (m == 1 || p <= r.plog[0][0]) { o.v = lnk_at(r.plog[0], o.dT); return o; }
    if (p >= r.plog[m - 1][0]) { o.v = lnk_at(r.plog[m - 1], o.dT); return o; }
    size_t i = 0;
    while (!(p < r.plog[i + 1][0])) ++i;     // P_i <= P < P_{i+1}
    S d1, d2;
    S l1 = lnk_at(r.plog[i], d1), l2 = lnk_at(r.plog[i + 1], d2);
    S lp1 = S(std::log(r.plog[i][0])), lp2 = S(std::log(r.plog[i + 1][0]));
    S slope = (l2 - l1) / (lp2 - lp1);
    S w = (log(P) - lp1) / (lp2 - lp1);
    o.v = l1 + slope * (log(P) - lp1);
    o.dT = d1 + w * (d2 - d1);
    o.dlnP = slope;
    return o;
}

// Chebyshev polynomials of the first kind T_0..T_{n-1} at x and their
// derivatives, from T_0 = 1, T_1 = x, T_{j+1} = 2 x T_j - T_{j-1}.
template <class S>
void cheb_poly(int n, S x, std::vector<S>& t, std::vector<S>& dt) {
    t.assign(n, S(0.0));
    dt.assign(n, S(0.0));
    t[0] = S(1.0);
    if (n > 1) { t[1] = x; dt[1] = S(1.0); }
    for (int j = 1; j + 1 < n; ++j) {
        t[j + 1] = S(2.0) * x * t[j] - t[j - 1];
        dt[j + 1] = S(2.0) * t[j] + S(2.0) * x * dt[j] - dt[j - 1];
    }
}

// Chebyshev: log10 k = sum_t sum_p a_tp T_t(Tr) T_p(Pr) with the reduced
// variables Tr = (2/T - 1/Tmin - 1/Tmax) / (1/Tmax - 1/Tmin) and
// Pr = (2 log10 P - log10 Pmin - log10 Pmax) / (log10 Pmax - log10 Pmin).
template <class S>
LnK<S> cheb_lnk(const Reaction& r, S T, S P) {
    const double iTmin = 1.0 / r.cheb_Tmin, iTmax = 1.0 / r.cheb_Tmax;
    const double lmin = std::log10(r.cheb_Pmin), lmax = std::log10(r.cheb_Pmax);
    S Tr = (S(2.0) / T - S(iTmin) - S(iTmax)) / S(iTmax - iTmin);
    S Prd = (S(2.0) * log10(P) - S(lmin) - S(lmax)) / S(lmax - lmin);
    std::vector<S> ft, dft, fp, dfp;
    cheb_poly(r.cheb_nt, Tr, ft, dft);
    cheb_poly(r.cheb_np, Prd, fp, dfp);
    S v(0.0), dv_dTr(0.0), dv_dPr(0.0);
    for (int t = 0; t < r.cheb_nt; ++t)
        for (int q = 0; q < r.cheb_np; ++q) {
            S a(r.cheb[(size_t)t * r.cheb_np + q]);
            v = v + a * ft[t] * fp[q];
            dv_dTr = dv_dTr + a * dft[t] * fp[q];
            dv_dPr = dv_dPr + a * ft[t] * dfp[q];
        }
    LnK<S> o;
    o.v = S(LN10) * v;
    // dTr/dT = -2 / (T^2 (1/Tmax - 1/Tmin)); dPr/d ln P = 2 / (ln 10 (log10 Pmax - log10 Pmin))
    o.dT = S(LN10) * dv_dTr * S(-2.0) / (T * T * S(iTmax - iTmin));
    o.dlnP = dv_dPr * S(2.0) / S(lmax - lmin);
    return o;
}

template <class S>
RxnEval<S> eval_reaction(const Mech& m, const Reaction& r, const State<S>& st,
                         const std::vector<Thermo<S>>& th, bool with_derivs,
                         const ParamShift<S>* shift = nullptr) {
    int ns = m.ns;
    RxnEval<S> e;
    S T = st.T;
    // the main Arrhenius expression ka: k_f itself, the high-pressure limit of
    // a falloff or chemically activated reaction, or a factor on a rate
    // constant tabulated in pressure
    S ka, dka_dT;
    if (shift) {
        S bb = S(r.b) + shift->b, tt = S(r.theta) + shift->theta;
        ka = exp(S(r.lnA) + shift->lnA + bb * log(T) - tt / T);
        dka_dT = ka * (bb / T + tt / (T * T));
    } else {
        ka = arrhenius(r.lnA, r.b, r.theta, T);
        if (!g_values_only) dka_dT = ka * (S(r.b) / T + S(r.theta) / (T * T));
    }
    S dlnk_dlnP(0.0);   // pressure dependence of k_f at fixed T (P-Log, Chebyshev)
    e.kf = ka;
    e.dkf_dT = dka_dT;
    if (r.pressure_table()) {
        LnK<S> t = r.type == T_PLOG ? plog_lnk(r, T, st.P) : cheb_lnk(r, T, st.P);
        S kt = exp(t.v);
        e.kf = ka * kt;
        if (!g_values_only) e.dkf_dT = dka_dT * kt + e.kf * t.dT;
        dlnk_dlnP = t.dlnP;
    }
    // falloff forms: the low-pressure limit; a chemically activated reaction's
    // rate multiplies it instead of the high-pressure limit
    S k0(0.0), dk0_dT(0.0);
    if (r.falloff()) {
        k0 = arrhenius(r.lnA0, r.b0, r.theta0, T);
        if (!g_values_only) dk0_dT = k0 * (S(r.b0) / T + S(r.theta0) / (T * T));
    }
    if (r.chemact) {
        e.kf = k0;
        e.dkf_dT = dk0_dT;
    }

    // reverse rate constant from the equilibrium constant:
    //   ln Kc = -sum_k nu_k G_k/(R T) + (sum_k nu_k) ln(P_ref / (R T))
    S sum_nu_g(0.0), sum_nu_dg(0.0);
    int sum_nu = 0;
    for (auto& p : r.reac) {
        sum_nu_g = sum_nu_g - S((double)p.second) * (th[p.first].h - th[p.first].s);
        if (!g_values_only) sum_nu_dg = sum_nu_dg - S((double)p.second) * (th[p.first].dh - th[p.first].ds);
        sum_nu -= p.second;
    }
    for (auto& p : r.prod) {
        sum_nu_g = sum_nu_g + S((double)p.second) * (th[p.first].h - th[p.first].s);
        if (!g_values_only) sum_nu_dg = sum_nu_dg + S((double)p.second) * (th[p.first].dh - th[p.first].ds);
        sum_nu += p.second;
    }
    if (r.rev) {
        S lnKc = -sum_nu_g + S((double)sum_nu) * log(S(PREF) / (S(RU) * T));
        S Kc = exp(lnKc);
        e.kr = e.kf / Kc;
        if (!g_values_only) {
            S dlnKc_dT = -sum_nu_dg - S((double)sum_nu) / T;
            e.dkr_dT = e.dkf_dT / Kc - e.kf * (Kc * dlnKc_dT) / (Kc * Kc);
        }
    } else {
        e.kr = S(0.0);
        e.dkr_dT = S(0.0);
    }

    e.Rf = e.kf * mass_action(r.reac, st.C);
    e.Rr = r.rev ? e.kr * mass_action(r.prod, st.C) : S(0.0);

    // pressure modification
    std::vector<double> alpha(ns, 1.0);
    for (auto& p : r.eff) alpha[p.first] = p.second;
    // third-body concentration [M] = C_tot + sum_k (alpha_k - 1) [C]_k with the
    // total concentration C_tot = P / (R T), a function of T and P only (equal
    // to sum_k alpha_k [C]_k; written this way, a species of default efficiency
    // does not enter [M] through the concentrations)
    S M(0.0);
    if (r.type == T_THREEBODY || r.falloff()) {
        M = st.P / (S(RU) * T);
        for (int k = 0; k < ns; ++k)
            if (alpha[k] != 1.0) M = M + S(alpha[k] - 1.0) * st.C[k];
    }

    e.dc_dC.assign(ns, S(0.0));
    e.dc_dCtot = S(0.0);
    e.dc_dT = S(0.0);
    S Pr_dc_dPr(0.0);   // Pr dc/dPr of a falloff reaction (Pr = k0 [M] / k_inf)
    if (r.type == T_ELEM || r.pressure_table()) {
        e.c = S(1.0);
    } else if (r.type == T_THREEBODY) {
        e.c = M;
        if (!g_values_only) {
            for (int k = 0; k < ns; ++k) e.dc_dC[k] = S(alpha[k] - 1.0);
            e.dc_dCtot = S(1.0);
        }
    } else {
        S Pr = k0 * M / ka;
        S dPr_dT(0.0);
        if (!g_values_only) dPr_dT = M * (dk0_dT * ka - k0 * dka_dT) / (ka * ka);
        S F(1.0), dF_dPr(0.0), dF_dT(0.0);
        if (r.type == T_TROE) {
            S Fcent = S(1.0 - r.alpha) * exp(-T / S(r.T3)) + S(r.alpha) * exp(-T / S(r.T1))
                      + exp(-S(r.T2) / T);
            S L = log10(Fcent);
            S cc = S(-0.4) - S(0.67) * L;
            S nn = S(0.75) - S(1.27) * L;
            S A = log10(Pr) + cc;
            S B = nn - S(0.14) * A;
            S f = A / B;
            S expo = L / (S(1.0) + f * f);       // log10 F
            F = exp(S(LN10) * expo);
            if (!g_values_only) {
            S dFcent_dT = -S(1.0 - r.alpha) / S(r.T3) * exp(-T / S(r.T3))
                          - S(r.alpha) / S(r.T1) * exp(-T / S(r.T1))
                          + S(r.T2) / (T * T) * exp(-S(r.T2) / T);
            // d f / d log10(Pr) and d f / d L
            S df_dlP = (B - A * S(-0.14)) / (B * B);
            S dA_dL = S(-0.67);
            S dB_dL = S(-1.27) - S(0.14) * dA_dL;
            S df_dL = (dA_dL * B - A * dB_dL) / (B * B);
            S dexpo_df = -L * S(2.0) * f / ((S(1.0) + f * f) * (S(1.0) + f * f));
            S dexpo_dL = S(1.0) / (S(1.0) + f * f) + dexpo_df * df_dL;
            // dF/dPr = F ln10 dexpo/df df/dlP dlP/dPr, dlP/dPr = 1/(Pr ln10)
            dF_dPr = F * dexpo_df * df_dlP / Pr;
            // dF/dT at fixed Pr, through Fcent: dL/dT = dFcent/dT / (Fcent ln10)
            dF_dT = F * S(LN10) * dexpo_dL * dFcent_dT / (Fcent * S(LN10));
            }
        } else if (r.type == T_SRI) {
            // SRI: F = d (a exp(-b/T) + exp(-T/c))^X T^e, X = 1 / (1 + (log10 Pr)^2)
            S a(r.sri[0]), b(r.sri[1]), cc(r.sri[2]), d(r.sri[3]), ee(r.sri[4]);
            S lP = log10(Pr);
            S X = S(1.0) / (S(1.0) + lP * lP);
            S base = a * exp(-b / T) + exp(-T / cc);
            F = d * exp(X * log(base)) * exp(ee * log(T));
            if (!g_values_only) {
                S dbase_dT = a * b / (T * T) * exp(-b / T) - exp(-T / cc) / cc;
                // dX/dPr = -2 log10(Pr) X^2 / (Pr ln 10)
                dF_dPr = F * log(base) * (S(-2.0) * lP * X * X) / (Pr * S(LN10));
                dF_dT = F * (X * dbase_dT / base + ee / T);
            }
        }
        S dc_dPr;
        if (r.chemact) {
            // chemically activated: c = F / (1 + Pr) on the rate with k_0
            e.c = F / (S(1.0) + Pr);
            if (!g_values_only) {
                dc_dPr = dF_dPr / (S(1.0) + Pr) - F / ((S(1.0) + Pr) * (S(1.0) + Pr));
                e.dc_dT = dc_dPr * dPr_dT + dF_dT / (S(1.0) + Pr);
            }
        } else {
            // c = F Pr / (1 + Pr), written as F / (1 + 1/Pr): the same value, but its
            // complex-step derivative carries no cancellation when Pr >> 1
            e.c = F / (S(1.0) + S(1.0) / Pr);
            if (!g_values_only) {
                dc_dPr = F / ((S(1.0) + Pr) * (S(1.0) + Pr)) + Pr / (S(1.0) + Pr) * dF_dPr;
                e.dc_dT = dc_dPr * dPr_dT + Pr / (S(1.0) + Pr) * dF_dT;
            }
        }
        if (!g_values_only) {
            for (int k = 0; k < ns; ++k) e.dc_dC[k] = dc_dPr * k0 * S(alpha[k] - 1.0) / ka;
            e.dc_dCtot = dc_dPr * k0 / ka;
            Pr_dc_dPr = Pr * dc_dPr;
        }
    }
    e.q = e.c * (e.Rf - e.Rr);
    if (g_values_only) return e;
    // R = Rf - Rr is proportional to k_f (k_r = k_f / Kc), and k_f to the main
    // Arrhenius factor except for a chemically activated reaction (k_f = k_0);
    // for falloff forms c also depends on that factor through Pr, with
    // dPr/d ln k_inf = -Pr
    e.dq_dlnk = (r.chemact ? S(0.0) : e.q) - (r.falloff() ? (e.Rf - e.Rr) * Pr_dc_dPr : S(0.0));
    // explicit pressure dependence of k_f (k_r = k_f / Kc follows it)
    e.dq_dP = e.c * (e.Rf - e.Rr) * dlnk_dlnP / st.P;
    if (!with_derivs) return e;

    e.dRf_dC.assign(ns, S(0.0));
    e.dRr_dC.assign(ns, S(0.0));
    for (int k = 0; k < ns; ++k) {
        e.dRf_dC[k] = e.kf * mass_action_d(r.reac, st.C, k);
        if (r.rev) e.dRr_dC[k] = e.kr * mass_action_d(r.prod, st.C, k);
    }
    e.dRf_dT = e.dkf_dT * mass_action(r.reac, st.C);
    e.dRr_dT = r.rev ? e.dkr_dT * mass_action(r.prod, st.C) : S(0.0);
    e.dq_dC.assign(ns, S(0.0));
    for (int k = 0; k < ns; ++k)
        e.dq_dC[k] = e.dc_dC[k] * (e.Rf - e.Rr) + e.c * (e.dRf_dC[k] - e.dRr_dC[k]);
    e.dq_dCtot = e.dc_dCtot * (e.Rf - e.Rr);
    e.dq_dT = e.dc_dT * (e.Rf - e.Rr) + e.c * (e.dRf_dT - e.dRr_dT);
    return e;
}

template <class S>
int net_nu(const Reaction& r, int k) {
    int nu = 0;
    for (auto& p : r.reac) if (p.first == k) nu -= p.second;
    for (auto& p : r.prod) if (p.first == k) nu += p.second;
    return nu;
}

// ---------------------------------------------------------------------------
// source terms

template <class S>
struct Eval {
    State<S> st;
    std::vector<Thermo<S>> th;
    std::vector<RxnEval<S>> rx;
    std::vector<S> wdot;          // all Ns species
    std::vector<S> e, chat;       // H or U, Cp or Cv  (J/kmol, J/(kmol K))
    S N, D, Tdot, Omega, Sdot;
    std::vector<S> f;             // d Phi / dt
};

template <class S>
Eval<S> evaluate(const Mech& m, int form, const S* x, S param, bool with_derivs,
                 const std::vector<ParamShift<S>>* shift = nullptr, bool frozen = false) {
    Eval<S> ev;
    int ns = m.ns, nr = (int)m.rx.size();
    ev.st = make_state(m, form, x, param, frozen);
    S T = ev.st.T;
    ev.th.resize(ns);
    for (int k = 0; k < ns; ++k) ev.th[k] = species_thermo(m.sp[k], T);
    ev.rx.resize(nr);
    for (int i = 0; i < nr; ++i)
        ev.rx[i] = eval_reaction(m, m.rx[i], ev.st, ev.th, with_derivs, shift ? &(*shift)[i] : nullptr);

    ev.wdot.assign(ns, S(0.0));
    for (int k = 0; k < ns; ++k)
        for (int i = 0; i < nr; ++i) {
            int nu = net_nu<S>(m.rx[i], k);
            if (nu) ev.wdot[k] = ev.wdot[k] + S((double)nu) * ev.rx[i].q;
        }

    // temperature source term: dT/dt = -sum_k e_k wdot_k / sum_k [C]_k chat_k
    ev.e.resize(ns);
    ev.chat.resize(ns);
    for (int k = 0; k < ns; ++k) {
        S H = S(RU) * T * ev.th[k].h;
        S Cp = S(RU) * ev.th[k].cp;
        if (form == FORM_CONP) { ev.e[k] = H; ev.chat[k] = Cp; }
        else { ev.e[k] = H - S(RU) * T; ev.chat[k] = Cp - S(RU); }
    }
    ev.N = S(0.0);
    ev.D = S(0.0);
    for (int k = 0; k < ns; ++k) {
        ev.N = ev.N + ev.e[k] * ev.wdot[k];
        ev.D = ev.D + ev.st.C[k] * ev.chat[k];
    }
    ev.Tdot = -ev.N / ev.D;

    // volume / pressure source term from d(PV = nRT)/dt with the bath gas
    // closed by conservation of mass: dn_Ns/dt = -sum_{k<Ns} W_k/W_Ns dn_k/dt
    double Wb = m.sp[ns - 1].W;
    ev.Omega = S(0.0);
    for (int k = 0; k < ns - 1; ++k)
        ev.Omega = ev.Omega + S(1.0 - m.sp[k].W / Wb) * ev.wdot[k];
    if (form == FORM_CONP)
        ev.Sdot = ev.st.V * ev.Tdot / T + ev.st.V * S(RU) * T * ev.Omega / ev.st.P;
    else
        ev.Sdot = ev.st.P * ev.Tdot / T + S(RU) * T * ev.Omega;

    ev.f.resize(ns + 1);
    ev.f[0] = ev.Tdot;
    ev.f[1] = ev.Sdot;
    for (int k = 0; k < ns - 1; ++k) ev.f[2 + k] = ev.st.V * ev.wdot[k];
    return ev;
}

// ---------------------------------------------------------------------------
// analytical Jacobian J[i][j] = d(dPhi_i/dt)/dPhi_j (Sec. 2.2), by the chain
// rule through the concentrations.

template <class S>
void jacobian(const Mech& m, int form, const S* x, S param, S* J, bool approx = false) {
    int ns = m.ns, nr = (int)m.rx.size(), N = ns + 1, bath = ns - 1;
    Eval<S> ev = evaluate(m, form, x, param, true);
    const State<S>& st = ev.st;
    S T = st.T, V = st.V, P = st.P;

    // dC[k][j] = d[C]_k / dPhi_j; nz marks the entries that are not
    // identically zero (the others are skipped in the chain rule below).
    std::vector<S> dC((size_t)ns * N, S(0.0));
    std::vector<char> nz((size_t)ns * N, 0);
    auto set = [&](int k, int j, S v) { dC[(size_t)k * N + j] = v; nz[(size_t)k * N + j] = 1; };
    auto dc = [&](int k, int j) -> S { return dC[(size_t)k * N + j]; };
    S sumC(0.0);
    for (int k = 0; k < ns - 1; ++k) sumC = sumC + st.C[k];
    set(bath, 0, -(P / (S(RU) * T)) / T);
    if (form == FORM_CONP) {
        for (int k = 0; k < ns - 1; ++k) set(k, 1, -st.C[k] / V);
        set(bath, 1, sumC / V);
    } else {
        set(bath, 1, S(1.0) / (S(RU) * T));
    }
    for (int j = 0; j < ns - 1; ++j) {
        set(j, 2 + j, S(1.0) / V);
        if (!approx) set(bath, 2 + j, -S(1.0) / V);
    }

    // dq_i/dPhi_j = sum_k dq_i/d[C]_k d[C]_k/dPhi_j (+ dq_i/dT at fixed [C] for j = T),
    // the sum taken over the k whose sensitivity is not identically zero
    std::vector<std::vector<int>> colnz(N);
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < ns; ++k)
            if (nz[(size_t)k * N + j]) colnz[j].push_back(k);
    // dC_tot/dPhi_j, C_tot = P / (R T): T and, for CONV, P
    std::vector<S> dCtot(N, S(0.0));
    dCtot[0] = -(P / (S(RU) * T)) / T;
    if (form == FORM_CONV) dCtot[1] = S(1.0) / (S(RU) * T);
    std::vector<S> dq((size_t)nr * N, S(0.0));
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < N; ++j) {
            S acc = (j == 0) ? ev.rx[i].dq_dT : S(0.0);
            for (int k : colnz[j]) acc = acc + ev.rx[i].dq_dC[k] * dc(k, j);
            if (j < 2) acc = acc + ev.rx[i].dq_dCtot * dCtot[j];
            // a rate constant tabulated in pressure: P is a state variable of CONV
            if (j == 1 && form == FORM_CONV) acc = acc + ev.rx[i].dq_dP;
            dq[(size_t)i * N + j] = acc;
        }

    // dwdot_k/dPhi_j for every species, bath gas included
    std::vector<S> dw((size_t)ns * N, S(0.0));
    for (int k = 0; k < ns; ++k)
        for (int i = 0; i < nr; ++i) {
            int nu = net_nu<S>(m.rx[i], k);
            if (!nu) continue;
            for (int j = 0; j < N; ++j)
                dw[(size_t)k * N + j] = dw[(size_t)k * N + j] + S((double)nu) * dq[(size_t)i * N + j];
        }

    // temperature row
    std::vector<S> dTdot(N);
    for (int j = 0; j < N; ++j) {
        S dN(0.0), dD(0.0);
        for (int k = 0; k < ns; ++k) {
            dN = dN + ev.e[k] * dw[(size_t)k * N + j];
            if (nz[(size_t)k * N + j]) dD = dD + ev.chat[k] * dc(k, j);
        }
        if (j == 0) {
            for (int k = 0; k < ns; ++k) {
                // de_k/dT from the polynomial: H = R T h(T) -> dH/dT = R (h + T dh/dT);
                // U = H - R T -> dU/dT = dH/dT - R.  dchat_k/dT = R dcp/dT.
                S dH = S(RU) * (ev.th[k].h + T * ev.th[k].dh);
                S de = (form == FORM_CONP) ? dH : dH - S(RU);
                dN = dN + de * ev.wdot[k];
                dD = dD + st.C[k] * S(RU) * ev.th[k].dcp;
            }
        }
        dTdot[j] = -(dN * ev.D - ev.N * dD) / (ev.D * ev.D);
    }

    // Omega = sum_{k<Ns} (1 - W_k/W_Ns) wdot_k
    double Wb = m.sp[bath].W;
    std::vector<S> dOm(N, S(0.0));
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < ns - 1; ++k)
            dOm[j] = dOm[j] + S(1.0 - m.sp[k].W / Wb) * dw[(size_t)k * N + j];

    for (int j = 0; j < N; ++j) {
        S dT_j = (j == 0) ? S(1.0) : S(0.0);
        S dS_j = (j == 1) ? S(1.0) : S(0.0);
        J[0 * N + j] = dTdot[j];
        if (form == FORM_CONP) {
            // dV/dt = V Tdot / T + V R T Omega / P
            J[1 * N + j] = dS_j * (ev.Tdot / T + S(RU) * T * ev.Omega / P)
                           + V * (dTdot[j] / T - ev.Tdot * dT_j / (T * T))
                           + V * S(RU) * (dT_j * ev.Omega + T * dOm[j]) / P;
        } else {
            // dP/dt = P Tdot / T + R T Omega
            J[1 * N + j] = dS_j * ev.Tdot / T
                           + P * (dTdot[j] / T - ev.Tdot * dT_j / (T * T))
                           + S(RU) * (dT_j * ev.Omega + T * dOm[j]);
        }
        for (int k = 0; k < ns - 1; ++k) {
            // dn_k/dt = V wdot_k
            S dV_j = (form == FORM_CONP && j == 1) ? S(1.0) : S(0.0);
            J[(2 + k) * N + j] = V * dw[(size_t)k * N + j] + dV_j * ev.wdot[k];
        }
    }
}


// ---------------------------------------------------------------------------
// adjoint: J^T v and the derivatives of v . dPhi/dt with respect to the
// Arrhenius parameters, one state.  dPhi/dt depends on reaction i's
// parameters only through q_i, so
//   d(v . f)/d theta_i = lambda_i dq_i/d theta_i,   lambda_i = v . df/dq_i,
// where df/dq_i follows from the source terms with dwdot_k/dq_i = nu_ki:
//   dTdot/dq_i = -dE_i / D,  dE_i = sum_k nu_ki e_k (all species),
//   dOmega/dq_i = sum_{k<Ns} (1 - W_k/W_Ns) nu_ki,
//   CONP dSdot/dq_i = V/T dTdot/dq_i + V R T/P dOmega/dq_i,
//   CONV dSdot/dq_i = P/T dTdot/dq_i + R T dOmega/dq_i,
//   d(dn_k/dt)/dq_i = V nu_ki,
// and dq_i/d ln A = dq_i/d ln k_f, dq_i/db = ln T dq_i/d ln k_f,
// dq_i/d(Ea/R) = -dq_i/d ln k_f / T.

template <class S>
void param_grad(const Mech& m, int form, const S* x, S param, const double* v, S* g /* [3][nr] */) {
    int ns = m.ns, nr = (int)m.rx.size();
    Eval<S> ev = evaluate(m, form, x, param, false);
    S T = ev.st.T, V = ev.st.V, P = ev.st.P;
    double Wb = m.sp[ns - 1].W;
    for (int i = 0; i < nr; ++i) {
        const Reaction& r = m.rx[i];
        S dE(0.0), dOm(0.0), vn(0.0);
        for (int k = 0; k < ns; ++k) {
            int nu = net_nu<S>(r, k);
            if (!nu) continue;
            dE = dE + S((double)nu) * ev.e[k];
            if (k < ns - 1) {
                dOm = dOm + S((1.0 - m.sp[k].W / Wb) * nu);
                vn = vn + S(v[2 + k] * nu);
            }
        }
        S dTdot = -dE / ev.D;
        S dSdot = (form == FORM_CONP) ? V / T * dTdot + V * S(RU) * T / P * dOm
                                      : P / T * dTdot + S(RU) * T * dOm;
        S lam = S(v[0]) * dTdot + S(v[1]) * dSdot + V * vn;
        S gl = lam * ev.rx[i].dq_dlnk;
        g[i] = gl;
        g[nr + i] = gl * log(T);
        g[2 * nr + i] = -gl / T;
    }
}

template <class S>
void jtv(const Mech& m, int form, const S* x, S param, const double* v, S* out) {
    int N = m.ns + 1;
    std::vector<S> J((size_t)N * N);
    jacobian(m, form, x, param, J.data());
    for (int j = 0; j < N; ++j) {
        S acc(0.0);
        for (int i = 0; i < N; ++i) acc = acc + J[(size_t)i * N + j] * S(v[i]);
        out[j] = acc;
    }
}

// ---------------------------------------------------------------------------
// structural sparsity pattern (Sec. 3.4): the temperature and state-parameter
// rows and columns are dense; species row k has column j when some reaction
// with a non-zero net coefficient of k has a rate of progress that depends on
// [C]_j (j a reactant, a product of a reversible reaction, or a third body
// with an efficiency other than the bath gas's); a rate that depends on the
// bath gas makes the row dense.  The diagonal is always present.

void pattern(const Mech& m, unsigned char* P, bool approx = false) {
    int ns = m.ns, N = ns + 1, bath = ns - 1;
    std::memset(P, 0, (size_t)N * N);
    for (int j = 0; j < N; ++j) { P[0 * N + j] = 1; P[1 * N + j] = 1; P[j * N + 0] = 1; P[j * N + 1] = 1; P[j * N + j] = 1; }
    for (const Reaction& r : m.rx) {
        std::vector<char> dep(ns, 0);
        for (auto& p : r.reac) dep[p.first] = 1;
        if (r.rev) for (auto& p : r.prod) dep[p.first] = 1;
        if (r.type != T_ELEM) {
            std::vector<double> alpha(ns, 1.0);
            for (auto& p : r.eff) alpha[p.first] = p.second;
            // exact: d[M]/dn_k = (alpha_k - alpha_Ns)/V; approximate: (alpha_k - 1)/V
            for (int k = 0; k < ns; ++k) if (alpha[k] != (approx ? 1.0 : alpha[bath])) dep[k] = 1;
            if (alpha[bath] != 1.0) dep[bath] = 1;
        }
        for (int k = 0; k < ns - 1; ++k) {
            if (net_nu<double>(r, k) == 0) continue;
            for (int j = 0; j < ns - 1; ++j)
                if (dep[j] || (dep[bath] && !approx)) P[(size_t)(2 + k) * N + 2 + j] = 1;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface (ctypes)

extern "C" {

void* ora_load(const char* path) {
    Mech* m = new Mech();
    if (!parse(path, *m)) { delete m; return nullptr; }
    return m;
}

void ora_free(void* h) { delete static_cast<Mech*>(h); }

int ora_ns(void* h) { return static_cast<Mech*>(h)->ns; }
int ora_nr(void* h) { return (int)static_cast<Mech*>(h)->rx.size(); }

void ora_thermo(void* h, int k, double T, double* out /* cp, h, s, dcp, dh, ds */) {
    const Mech& m = *static_cast<Mech*>(h);
    Thermo<double> t = species_thermo(m.sp[k], T);
    out[0] = t.cp; out[1] = t.h; out[2] = t.s; out[3] = t.dcp; out[4] = t.dh; out[5] = t.ds;
}

// Sub-components at one state: per reaction kf, kr, c, Rf, Rr, q (6*nr),
// then wdot (ns), then C (ns), then (Tdot, Sdot, N, D, Omega).
void ora_components(void* h, int form, const double* x, double param, double* out) {
    const Mech& m = *static_cast<Mech*>(h);
    Eval<double> ev = evaluate(m, form, x, param, false);
    int nr = (int)m.rx.size(), ns = m.ns;
    for (int i = 0; i < nr; ++i) {
        const RxnEval<double>& r = ev.rx[i];
        double* o = out + 6 * i;
        o[0] = r.kf; o[1] = r.kr; o[2] = r.c; o[3] = r.Rf; o[4] = r.Rr; o[5] = r.q;
    }
    for (int k = 0; k < ns; ++k) out[6 * nr + k] = ev.wdot[k];
    for (int k = 0; k < ns; ++k) out[6 * nr + ns + k] = ev.st.C[k];
    double* t = out + 6 * nr + 2 * ns;
    t[0] = ev.Tdot; t[1] = ev.Sdot; t[2] = ev.N; t[3] = ev.D; t[4] = ev.Omega;
}

// Source terms for n states, state rows of length N (row-major); bound (if
// not NULL) receives the running error bound of each value, u * m, in the
// value's units.
void ora_source(void* h, int form, long n, const double* x, const double* param,
                double* f, double* bound) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    for (long s = 0; s < n; ++s) {
        const double* xs = x + s * N;
        if (bound) {
            std::vector<Err> xx(N);
            for (int i = 0; i < N; ++i) xx[i] = Err(xs[i]);
            Eval<Err> ev = evaluate(m, form, xx.data(), Err(param[s]), false);
            for (int i = 0; i < N; ++i) { f[s * N + i] = ev.f[i].v; bound[s * N + i] = U_ROUND * ev.f[i].m; }
        } else {
            Eval<double> ev = evaluate(m, form, xs, param[s], false);
            for (int i = 0; i < N; ++i) f[s * N + i] = ev.f[i];
        }
    }
}

// Analytical Jacobian, dense row-major N*N per state, optional running error
// bounds; approx != 0: the approximate form.
void ora_jacobian_ex(void* h, int form, long n, const double* x, const double* param,
                     double* J, double* bound, int approx) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    size_t NN = (size_t)N * N;
    for (long s = 0; s < n; ++s) {
        const double* xs = x + s * N;
        if (bound) {
            std::vector<Err> xx(N), JJ(NN);
            for (int i = 0; i < N; ++i) xx[i] = Err(xs[i]);
            jacobian(m, form, xx.data(), Err(param[s]), JJ.data(), approx != 0);
            for (size_t e = 0; e < NN; ++e) { J[s * NN + e] = JJ[e].v; bound[s * NN + e] = U_ROUND * JJ[e].m; }
        } else {
            jacobian(m, form, xs, param[s], J + s * NN, approx != 0);
        }
    }
}

void ora_jacobian(void* h, int form, long n, const double* x, const double* param, double* J, double* bound) {
    ora_jacobian_ex(h, form, n, x, param, J, bound, 0);
}

// The same definitions in long double (64-bit significand), rounded to
// double at the end: a reference about 2^11 times more precise than the
// double evaluation, used to check the running error bounds.
void ora_source_ld(void* h, int form, long n, const double* x, const double* param, double* f) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    for (long s = 0; s < n; ++s) {
        std::vector<long double> xx(N);
        for (int i = 0; i < N; ++i) xx[i] = x[s * N + i];
        Eval<long double> ev = evaluate(m, form, xx.data(), (long double)param[s], false);
        for (int i = 0; i < N; ++i) f[s * N + i] = (double)ev.f[i];
    }
}

void ora_jacobian_ld(void* h, int form, long n, const double* x, const double* param, double* J, int approx) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    size_t NN = (size_t)N * N;
    for (long s = 0; s < n; ++s) {
        std::vector<long double> xx(N), JJ(NN);
        for (int i = 0; i < N; ++i) xx[i] = x[s * N + i];
        jacobian(m, form, xx.data(), (long double)param[s], JJ.data(), approx != 0);
        for (size_t e = 0; e < NN; ++e) J[s * NN + e] = (double)JJ[e];
    }
}

// Arithmetic operations of the source terms of one state as the definitions
// above write them: out = {+ - * / count, exp count, log count, log10 count}.
// f: the source terms of that evaluation (N values), which must equal
// ora_source's.
void ora_source_ops(void* h, int form, const double* x, double param, double* out, double* f) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    std::vector<Cnt> xx(N);
    for (int i = 0; i < N; ++i) xx[i] = Cnt(x[i]);
    g_ops = OpCount();
    g_values_only = true;
    Eval<Cnt> ev = evaluate(m, form, xx.data(), Cnt(param), false);
    g_values_only = false;
    out[0] = g_ops.flops;
    out[1] = g_ops.exps;
    out[2] = g_ops.logs;
    out[3] = g_ops.log10s;
    if (f)
        for (int i = 0; i < N; ++i) f[i] = ev.f[i].v;
}

// Complex-step Jacobian: column j = Im f(Phi + i h_j e_j) / h_j with
// h_j = hrel * max(|Phi_j|, 1e-300).
void ora_jacobian_cs_ex(void* h, int form, long n, const double* x, const double* param,
                        double hrel, double* J, int approx) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    typedef std::complex<double> C;
    for (long s = 0; s < n; ++s) {
        const double* xs = x + s * N;
        for (int j = 0; j < N; ++j) {
            std::vector<C> xx(N);
            for (int i = 0; i < N; ++i) xx[i] = C(xs[i], 0.0);
            double hj = hrel * std::fmax(std::fabs(xs[j]), 1e-300);
            xx[j] = C(xs[j], hj);
            Eval<C> ev = evaluate<C>(m, form, xx.data(), C(param[s], 0.0), false, nullptr, approx != 0);
            for (int i = 0; i < N; ++i) J[(size_t)s * N * N + (size_t)i * N + j] = ev.f[i].imag() / hj;
        }
    }
}

void ora_jacobian_cs(void* h, int form, long n, const double* x, const double* param, double hrel, double* J) {
    ora_jacobian_cs_ex(h, form, n, x, param, hrel, J, 0);
}

// Central finite-difference Jacobian with step h_j = rel * max(|Phi_j|, 1e-300).
void ora_jacobian_fd(void* h, int form, long n, const double* x, const double* param,
                     double rel, double* J) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    for (long s = 0; s < n; ++s) {
        const double* xs = x + s * N;
        for (int j = 0; j < N; ++j) {
            std::vector<double> xp(xs, xs + N), xm(xs, xs + N);
            double hj = rel * std::fmax(std::fabs(xs[j]), 1e-300);
            xp[j] += hj;
            xm[j] -= hj;
            Eval<double> ep = evaluate(m, form, xp.data(), param[s], false);
            Eval<double> em = evaluate(m, form, xm.data(), param[s], false);
            for (int i = 0; i < N; ++i)
                J[(size_t)s * N * N + (size_t)i * N + j] = (ep.f[i] - em.f[i]) / (xp[j] - xm[j]);
        }
    }
}

void ora_pattern(void* h, unsigned char* P) { pattern(*static_cast<Mech*>(h), P); }
void ora_pattern_ex(void* h, unsigned char* P, int approx) { pattern(*static_cast<Mech*>(h), P, approx != 0); }

// Adjoint over n states (rows of length N, v likewise): jtv[s] = J(s)^T v[s];
// grad[3][nr] = sum over states of d(v . dPhi/dt)/d(ln A, b, Ea/R) per reaction
// in description order.  Optional running error bounds of both.
void ora_adjoint(void* h, int form, long n, const double* x, const double* param, const double* v,
                 double* jtv_out, double* grad, double* jtv_scale, double* grad_scale) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1, nr = (int)m.rx.size();
    std::vector<Err> gsum(3 * nr, Err(0.0));
    std::vector<double> gd(3 * nr, 0.0);
    for (long s = 0; s < n; ++s) {
        const double* xs = x + s * N;
        const double* vs = v + s * N;
        if (jtv_scale || grad_scale) {
            std::vector<Err> xx(N), o(N), g(3 * nr);
            for (int i = 0; i < N; ++i) xx[i] = Err(xs[i]);
            jtv(m, form, xx.data(), Err(param[s]), vs, o.data());
            for (int j = 0; j < N; ++j) {
                jtv_out[s * N + j] = o[j].v;
                if (jtv_scale) jtv_scale[s * N + j] = U_ROUND * o[j].m;
            }
            param_grad(m, form, xx.data(), Err(param[s]), vs, g.data());
            for (int q = 0; q < 3 * nr; ++q) gsum[q] = gsum[q] + g[q];
        } else {
            std::vector<double> g(3 * nr);
            jtv(m, form, xs, param[s], vs, jtv_out + s * N);
            param_grad(m, form, xs, param[s], vs, g.data());
            for (int q = 0; q < 3 * nr; ++q) gd[q] += g[q];
        }
    }
    for (int q = 0; q < 3 * nr; ++q) {
        grad[q] = (jtv_scale || grad_scale) ? gsum[q].v : gd[q];
        if (grad_scale) grad_scale[q] = U_ROUND * gsum[q].m;
    }
}

// Complex-step parameter derivatives: for every reaction and parameter,
// Im(v . f(theta + i h)) / h summed over states, h = hrel * max(|theta|, 1).
void ora_param_grad_cs(void* h, int form, long n, const double* x, const double* param,
                       const double* v, double hrel, double* grad) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1, nr = (int)m.rx.size();
    typedef std::complex<double> C;
    for (int q = 0; q < 3 * nr; ++q) grad[q] = 0.0;
    for (long s = 0; s < n; ++s) {
        std::vector<C> xx(N);
        for (int i = 0; i < N; ++i) xx[i] = C(x[s * N + i], 0.0);
        for (int i = 0; i < nr; ++i) {
            const Reaction& r = m.rx[i];
            const double base[3] = {r.lnA, r.b, r.theta};
            for (int a = 0; a < 3; ++a) {
                std::vector<ParamShift<C>> sh(nr, ParamShift<C>{C(0.0), C(0.0), C(0.0)});
                double hh = hrel * std::fmax(std::fabs(base[a]), 1.0);
                C d(0.0, hh);
                if (a == 0) sh[i].lnA = d; else if (a == 1) sh[i].b = d; else sh[i].theta = d;
                Eval<C> ev = evaluate(m, form, xx.data(), C(param[s], 0.0), false, &sh);
                double acc = 0.0;
                for (int k = 0; k < N; ++k) acc += v[s * N + k] * ev.f[k].imag() / hh;
                grad[a * nr + i] += acc;
            }
        }
    }
}

// Complex-step directional derivative: out[s] = Im f(Phi_s + i h u_s) / h = J(s) u_s.
void ora_jvp_cs(void* h, int form, long n, const double* x, const double* param, const double* u,
                double hstep, double* out) {
    const Mech& m = *static_cast<Mech*>(h);
    int N = m.ns + 1;
    typedef std::complex<double> C;
    for (long s = 0; s < n; ++s) {
        std::vector<C> xx(N);
        for (int i = 0; i < N; ++i) xx[i] = C(x[s * N + i], hstep * u[s * N + i]);
        Eval<C> ev = evaluate(m, form, xx.data(), C(param[s], 0.0), false);
        for (int i = 0; i < N; ++i) out[s * N + i] = ev.f[i].imag() / hstep;
    }
}

}  // extern "C"
