// Host mechanism compiler: parse and validate a mechanism description, derive
// the Jacobian's CSR pattern (paper Sec. 3.4) and the static scatter tables
// that replace the paper's run-time linear search of a CSR row (Sec. 3.4,
// sparse index lookup), and upload everything to the device once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "internal.h"

namespace pj {

namespace {

// ---------------------------------------------------------------------------
// description parsing (one whitespace-separated token stream)

struct Tokens {
    std::vector<std::string> t;
    size_t p = 0;
    bool more() const { return p < t.size(); }
    const std::string& peek() const { static std::string e; return p < t.size() ? t[p] : e; }
    bool word(std::string& s) { if (p >= t.size()) return false; s = t[p++]; return true; }
    bool integer(long& v) {
        if (p >= t.size()) return false;
        char* end = nullptr;
        v = std::strtol(t[p].c_str(), &end, 10);
        if (!end || *end) return false;
        ++p;
        return true;
    }
    bool real(double& v) {
        if (p >= t.size()) return false;
        char* end = nullptr;
        v = std::strtod(t[p].c_str(), &end);
        if (!end || *end) return false;
        ++p;
        return true;
    }
    bool expect(const char* w) { std::string s; return word(s) && s == w; }
};

pj_status parse_description(const char* path, Mechanism& m, std::string& err) {
    std::ifstream f(path);
    if (!f) { err = std::string("cannot open ") + path; return PJ_E_INVALID; }
    Tokens tk;
    std::string w;
    while (f >> w) tk.t.push_back(w);
    long v;
    if (!tk.expect("PJMECH") || !tk.integer(v) || v != 1) { err = "not a PJMECH 1 description"; return PJ_E_PARSE; }
    if (!tk.expect("SPECIES") || !tk.integer(v) || v < 2 || v > 60000) { err = "bad SPECIES record"; return PJ_E_PARSE; }
    m.ns = (int)v;
    m.W.resize(m.ns);
    m.comp.resize((size_t)m.ns * 4);
    m.tmid.resize(m.ns);
    m.alo.resize((size_t)m.ns * 7);
    m.ahi.resize((size_t)m.ns * 7);
    for (int k = 0; k < m.ns; ++k) {
        std::string name;
        double tl, th;
        if (!tk.expect("SP") || !tk.integer(v) || v != k || !tk.word(name) || !tk.real(m.W[k])) {
            err = "bad SP record " + std::to_string(k);
            return PJ_E_PARSE;
        }
        for (int e = 0; e < 4; ++e) {
            if (!tk.integer(v) || v < 0) { err = "bad composition of species " + std::to_string(k); return PJ_E_PARSE; }
            m.comp[(size_t)k * 4 + e] = (int)v;
        }
        if (!tk.real(tl) || !tk.real(m.tmid[k]) || !tk.real(th)) { err = "bad temperature ranges"; return PJ_E_PARSE; }
        for (int c = 0; c < 7; ++c) if (!tk.real(m.alo[(size_t)k * 7 + c])) { err = "bad NASA coefficients"; return PJ_E_PARSE; }
        for (int c = 0; c < 7; ++c) if (!tk.real(m.ahi[(size_t)k * 7 + c])) { err = "bad NASA coefficients"; return PJ_E_PARSE; }
        if (!(m.W[k] > 0) || !(m.tmid[k] > 0)) { err = "non-positive weight or T_mid"; return PJ_E_PARSE; }
    }
    if (!tk.expect("REACTIONS") || !tk.integer(v) || v < 0 || v > 1000000) { err = "bad REACTIONS record"; return PJ_E_PARSE; }
    m.nr = (int)v;
    m.rx.resize(m.nr);
    for (int i = 0; i < m.nr; ++i) {
        Mechanism::Rxn& r = m.rx[i];
        std::string kind;
        long rev, n;
        if (!tk.expect("RX") || !tk.integer(v) || v != i || !tk.word(kind) || !tk.integer(rev)) {
            err = "bad RX record " + std::to_string(i);
            return PJ_E_PARSE;
        }
        if (kind == "ELEM") r.kind = K_ELEM;
        else if (kind == "THREEBODY") r.kind = K_THREEBODY;
        else if (kind == "LINDEMANN") r.kind = K_LINDEMANN;
        else if (kind == "TROE") r.kind = K_TROE;
        else if (kind == "SRI") r.kind = K_SRI;
        else if (kind == "PLOG") r.kind = K_PLOG;
        else if (kind == "CHEB") r.kind = K_CHEB;
        else { err = "unknown reaction type " + kind; return PJ_E_PARSE; }
        r.rev = rev != 0;
        for (int side = 0; side < 2; ++side) {
            auto& lst = side == 0 ? r.reac : r.prod;
            if (!tk.integer(n) || n < 0 || n > 16) { err = "bad side of reaction " + std::to_string(i); return PJ_E_PARSE; }
            for (long a = 0; a < n; ++a) {
                long s, nu;
                if (!tk.integer(s) || !tk.integer(nu) || s < 0 || s >= m.ns || nu <= 0) {
                    err = "bad species/coefficient in reaction " + std::to_string(i);
                    return PJ_E_PARSE;
                }
                bool merged = false;
                for (auto& e : lst) if (e.first == s) { e.second += (int)nu; merged = true; }
                if (!merged) lst.push_back({(int)s, (int)nu});
            }
        }
        if (!tk.real(r.lnA) || !tk.real(r.b) || !tk.real(r.theta)) { err = "bad Arrhenius in reaction " + std::to_string(i); return PJ_E_PARSE; }
        bool has_low = false, has_troe = false, has_sri = false;
        auto keyword = [&](const std::string& k) {
            return k == "LOW" || k == "TROE" || k == "SRI" || k == "CHEMACT" || k == "PLOG" || k == "CHEB" || k == "EFF";
        };
        while (tk.more() && keyword(tk.peek())) {
            std::string kw;
            tk.word(kw);
            if (kw == "LOW") {
                if (!tk.real(r.lnA0) || !tk.real(r.b0) || !tk.real(r.theta0)) { err = "bad LOW"; return PJ_E_PARSE; }
                has_low = true;
            } else if (kw == "TROE") {
                if (!tk.real(r.alpha) || !tk.real(r.T3) || !tk.real(r.T1) || !tk.real(r.T2)) { err = "bad TROE"; return PJ_E_PARSE; }
                has_troe = true;
            } else if (kw == "SRI") {
                for (double& x : r.sri) if (!tk.real(x)) { err = "bad SRI"; return PJ_E_PARSE; }
                has_sri = true;
            } else if (kw == "CHEMACT") {
                r.chemact = true;
            } else if (kw == "PLOG") {
                if (!tk.integer(n) || n < 1) { err = "bad PLOG count"; return PJ_E_PARSE; }
                if (n > MAX_PLOG) { err = "more than " + std::to_string(MAX_PLOG) + " PLOG pressures"; return PJ_E_UNSUPPORTED; }
                for (long a = 0; a < n; ++a) {
                    std::array<double, 4> pt;
                    for (double& x : pt) if (!tk.real(x)) { err = "bad PLOG entry"; return PJ_E_PARSE; }
                    if (!(pt[0] > 0) || (a && !(pt[0] > r.plog.back()[0]))) { err = "PLOG pressures must be positive and ascending"; return PJ_E_PARSE; }
                    r.plog.push_back(pt);
                }
            } else if (kw == "CHEB") {
                long nt, np;
                if (!tk.integer(nt) || !tk.integer(np) || nt < 1 || np < 1) { err = "bad CHEB size"; return PJ_E_PARSE; }
                if (nt > MAX_CHEB || np > MAX_CHEB) {
                    err = "more than " + std::to_string(MAX_CHEB) + " CHEB coefficients in one direction";
                    return PJ_E_UNSUPPORTED;
                }
                r.cheb_nt = (int)nt;
                r.cheb_np = (int)np;
                if (!tk.real(r.cheb_T[0]) || !tk.real(r.cheb_T[1]) || !tk.real(r.cheb_P[0]) || !tk.real(r.cheb_P[1])) { err = "bad CHEB range"; return PJ_E_PARSE; }
                if (!(r.cheb_T[0] > 0 && r.cheb_T[1] > r.cheb_T[0] && r.cheb_P[0] > 0 && r.cheb_P[1] > r.cheb_P[0])) { err = "CHEB ranges must be positive and ascending"; return PJ_E_PARSE; }
                r.cheb.resize((size_t)nt * np);
                for (double& x : r.cheb) if (!tk.real(x)) { err = "bad CHEB coefficient"; return PJ_E_PARSE; }
            } else {
                if (!tk.integer(n) || n < 0) { err = "bad EFF"; return PJ_E_PARSE; }
                for (long a = 0; a < n; ++a) {
                    long s;
                    double al;
                    if (!tk.integer(s) || !tk.real(al) || s < 0 || s >= m.ns || al < 0) { err = "bad efficiency"; return PJ_E_PARSE; }
                    r.eff.push_back({(int)s, al});
                }
            }
        }
        if (kind_falloff(r.kind) != has_low) { err = "falloff reaction without LOW (or LOW on another type)"; return PJ_E_PARSE; }
        if ((r.kind == K_TROE) != has_troe) { err = "TROE parameters do not match the reaction type"; return PJ_E_PARSE; }
        if ((r.kind == K_SRI) != has_sri) { err = "SRI parameters do not match the reaction type"; return PJ_E_PARSE; }
        if (r.kind == K_TROE && (!(r.T3 > 0) || !(r.T1 > 0))) { err = "Troe T*** and T* must be positive"; return PJ_E_PARSE; }
        if (r.kind == K_SRI && (!(r.sri[0] >= 0) || !(r.sri[2] > 0) || !(r.sri[3] > 0))) { err = "SRI needs a >= 0, c > 0 and d > 0"; return PJ_E_PARSE; }
        if (r.chemact && !kind_falloff(r.kind)) { err = "CHEMACT on a reaction without a falloff form"; return PJ_E_PARSE; }
        if ((r.kind == K_PLOG) != !r.plog.empty()) { err = "PLOG table does not match the reaction type"; return PJ_E_PARSE; }
        if ((r.kind == K_CHEB) != !r.cheb.empty()) { err = "CHEB table does not match the reaction type"; return PJ_E_PARSE; }
        if ((r.kind == K_ELEM || kind_table(r.kind)) && !r.eff.empty()) { err = "efficiencies on a reaction without a third body"; return PJ_E_PARSE; }
    }
    if (!tk.expect("END") || tk.more()) { err = "missing END"; return PJ_E_PARSE; }
    return PJ_OK;
}

std::vector<std::pair<int, double>> enhanced(const Mechanism::Rxn& r) {
    std::map<int, double> a;
    for (auto& e : r.eff) a[e.first] = e.second;
    std::vector<std::pair<int, double>> out;
    for (auto& e : a) if (e.second != 1.0) out.push_back(e);
    return out;
}

pj_status validate(const Mechanism& m, std::string& err) {
    for (int i = 0; i < m.nr; ++i) {
        const auto& r = m.rx[i];
        if (r.reac.empty() || r.prod.empty()) { err = "empty reaction side in reaction " + std::to_string(i); return PJ_E_UNSUPPORTED; }
        if (r.reac.size() > MAXSIDE || r.prod.size() > MAXSIDE) {
            err = "more than 3 species on one side of reaction " + std::to_string(i);
            return PJ_E_UNSUPPORTED;
        }
        for (auto& a : r.reac) {
            if (a.second > 2) { err = "coefficient above 2 in reaction " + std::to_string(i); return PJ_E_UNSUPPORTED; }
            for (auto& b : r.prod)
                if (a.first == b.first) { err = "species on both sides of reaction " + std::to_string(i); return PJ_E_UNSUPPORTED; }
        }
        for (auto& b : r.prod)
            if (b.second > 2) { err = "coefficient above 2 in reaction " + std::to_string(i); return PJ_E_UNSUPPORTED; }
        if (enhanced(r).size() > (size_t)MAXEFF) {
            err = "more than " + std::to_string(MAXEFF) + " third-body efficiencies in reaction " + std::to_string(i);
            return PJ_E_UNSUPPORTED;
        }
        for (int e = 0; e < 4; ++e) {
            long lhs = 0, rhs = 0;
            for (auto& a : r.reac) lhs += (long)a.second * m.comp[(size_t)a.first * 4 + e];
            for (auto& b : r.prod) rhs += (long)b.second * m.comp[(size_t)b.first * 4 + e];
            if (lhs != rhs) { err = "reaction " + std::to_string(i) + " does not conserve elements"; return PJ_E_UNBALANCED; }
        }
    }
    return PJ_OK;
}

// third-body efficiencies different from one, merged per species
bool depends_on_bath(const Mechanism& m, const Mechanism::Rxn& r) {
    int bath = m.ns - 1;
    for (auto& a : r.reac) if (a.first == bath) return true;
    if (r.rev) for (auto& b : r.prod) if (b.first == bath) return true;
    if (r.kind != K_ELEM) for (auto& e : enhanced(r)) if (e.first == bath) return true;
    return false;
}

// The Jacobian pattern (Sec. 3.4).  Approximate form: no dense rows from the
// bath gas (its moles are held fixed against the other species').
void build_pattern(Mechanism& m) {
    int ns = m.ns, N = ns + 1, bath = ns - 1;
    const bool approx = (m.opts & PJ_OPT_APPROX_JACOBIAN) != 0;
    std::vector<std::vector<char>> P(N, std::vector<char>(N, 0));
    for (int i = 0; i < N; ++i) { P[0][i] = P[1][i] = P[i][0] = P[i][1] = P[i][i] = 1; }
    for (const auto& r : m.rx) {
        std::vector<int> deps;
        for (auto& a : r.reac) deps.push_back(a.first);
        if (r.rev) for (auto& b : r.prod) deps.push_back(b.first);
        if (r.kind != K_ELEM) for (auto& e : enhanced(r)) deps.push_back(e.first);
        bool dense = !approx && depends_on_bath(m, r);
        auto row = [&](int k) {
            if (k == bath) return;
            if (dense) { for (int j = 2; j < N; ++j) P[2 + k][j] = 1; return; }
            for (int j : deps) if (j != bath) P[2 + k][2 + j] = 1;
        };
        for (auto& a : r.reac) row(a.first);
        for (auto& b : r.prod) row(b.first);
    }
    m.row_ptr.assign(N + 1, 0);
    m.col_idx.clear();
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) if (P[i][j]) m.col_idx.push_back(j);
        m.row_ptr[i + 1] = (int32_t)m.col_idx.size();
    }
    m.nnz = (int)m.col_idx.size();
    // column order (CCS): rows ascending in each column
    m.col_ptr.assign(N + 1, 0);
    m.row_idx.clear();
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) if (P[i][j]) m.row_idx.push_back(i);
        m.col_ptr[j + 1] = (int32_t)m.row_idx.size();
    }
}

int csr_find(const Mechanism& m, int row, int col) {
    auto b = m.col_idx.begin() + m.row_ptr[row], e = m.col_idx.begin() + m.row_ptr[row + 1];
    auto it = std::lower_bound(b, e, col);
    return (it != e && *it == col) ? (int)(it - m.col_idx.begin()) : -1;
}

struct Section {
    size_t off;
    size_t bytes;
};

}  // namespace

pj_status build_mechanism(const char* path, Mechanism& m, std::string& err) {
    pj_status st = parse_description(path, m, err);
    if (st != PJ_OK) return st;
    st = validate(m, err);
    if (st != PJ_OK) return st;
    // Kernel order: by kind and reversibility, then by shape (number of
    // reactant and product species), so that the reactions a wave handles
    // together take the same branches and the empty slots of a 64-reaction
    // chunk are skipped by wave-uniform branches instead of masked execution.
    m.order.resize(m.nr);
    for (int i = 0; i < m.nr; ++i) m.order[i] = i;
    auto key = [&](int i) {
        const auto& r = m.rx[i];
        // elementary (reversible, irreversible), third-body, falloff
        // (Lindemann, Troe, SRI), chemically activated (same forms), P-Log,
        // Chebyshev
        int cls = r.kind == K_ELEM ? (r.rev ? 0 : 1)
                  : kind_falloff(r.kind) ? r.kind + 1 + (r.chemact ? 3 : 0)
                  : r.kind == K_THREEBODY ? 2 : r.kind + 4;
        return cls * 100 + (int)r.reac.size() * 10 + (int)r.prod.size();
    };
    std::stable_sort(m.order.begin(), m.order.end(), [&](int a, int b) { return key(a) < key(b); });
    build_pattern(m);
    if (m.nnz >= 65535) { err = "more than 65534 Jacobian non-zeros"; return PJ_E_UNSUPPORTED; }
    return PJ_OK;
}

pj_status upload_mechanism(Mechanism& m, std::string& err) {
    const int ns = m.ns, nr = m.nr, N = ns + 1, bath = ns - 1;
    const int nr_pad = std::max(64, (nr + 63) / 64 * 64);
    const double Wb = m.W[bath];

    // ---- species tables.  Coefficient layout of one range (c[]):
    //   0..4   Cp/R    = c0 + c1 T + c2 T^2 + c3 T^3 + c4 T^4
    //   5..8   H/RT    = c0 + c5 T + c6 T^2 + c7 T^3 + c8 T^4 + c12 / T
    //   9..11  S/R     = c0 ln T + c1 T + c9 T^2 + c10 T^3 + c11 T^4 + c13
    //   14..16 dCp/R/dT = c1 + c14 T + c15 T^2 + c16 T^3
    std::vector<ThermoRec> th((size_t)ns * 2);
    std::vector<double> tmid(ns), wfac(ns);
    for (int k = 0; k < ns; ++k) {
        for (int rg = 0; rg < 2; ++rg) {
            const double* a = (rg == 0 ? m.alo.data() : m.ahi.data()) + (size_t)k * 7;
            double row[TH_N] = {a[0], a[1], a[2], a[3], a[4],
                                a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5,
                                a[2] / 2, a[3] / 3, a[4] / 4,
                                a[5], a[6],
                                2 * a[2], 3 * a[3], 4 * a[4],
                                0.0};
            for (int c = 0; c < TH_N; ++c) th[(size_t)k * 2 + rg].c[c] = row[c];
        }
        tmid[k] = m.tmid[k];
        wfac[k] = k == bath ? 0.0 : 1.0 - m.W[k] / Wb;
    }

    // ---- reaction records (kernel order)
    std::vector<RxnRec> rec(nr_pad);
    std::vector<FallRec> fall(nr_pad);
    std::vector<JacRec> jrec(nr_pad);
    std::memset(rec.data(), 0, rec.size() * sizeof(RxnRec));
    std::memset(fall.data(), 0, fall.size() * sizeof(FallRec));
    std::memset(jrec.data(), 0xFF, jrec.size() * sizeof(JacRec));
    std::vector<EffRec> effrec(1);
    auto empty_eff = [&](EffRec& E) {
        std::memset(&E, 0, sizeof(E));
        std::memset(E.slot, 0xFF, sizeof(E.slot));
        for (int q = 0; q < MAXEFF; ++q) E.sp[q] = (uint16_t)ns;
    };
    empty_eff(effrec[0]);
    std::vector<char> dense_row(ns, 0);
    std::vector<TabRec> tabs;
    std::vector<double> tabd;
    // Slot positions.  The lanes of a wave handle 64 consecutive reactions
    // and scatter slot a of every reaction in the same instruction, so a
    // species that sits in the same slot of many of those reactions (a hub
    // such as a radical present in most reactions) makes the LDS serialise the
    // additions.  Within each side the order of the species is free: for every
    // chunk of 64 reactions choose, greedily, the arrangement that adds the
    // fewest repeats of an address already used at the same slot position.
    std::vector<std::array<int, NSLOT>> SPA(nr), NUA(nr);
    {
        // orders of the species of one side; species stay in the leading
        // positions so that a chunk of same-shape reactions leaves the same
        // trailing positions empty (skipped as a whole by the kernel)
        static const int perms[6][3] = {{0, 1, 2}, {1, 0, 2}, {0, 2, 1}, {2, 0, 1}, {1, 2, 0}, {2, 1, 0}};
        auto nperm = [](size_t n) { return n <= 1 ? 1 : n == 2 ? 2 : 6; };
        std::map<long, int> cnt;   // (position code, address) -> uses in this chunk
        auto code = [](int kind, int pos, long addr) { return ((long)kind << 56) | ((long)pos << 48) | addr; };
        for (int p = 0; p < nr; ++p) {
            if (p % 64 == 0) cnt.clear();
            const auto& r = m.rx[m.order[p]];
            int rs[3] = {ns, ns, ns}, rn[3] = {0, 0, 0}, ps[3] = {ns, ns, ns}, pn[3] = {0, 0, 0};
            for (size_t a = 0; a < r.reac.size(); ++a) { rs[a] = r.reac[a].first; rn[a] = r.reac[a].second; }
            for (size_t b = 0; b < r.prod.size(); ++b) { ps[b] = r.prod[b].first; pn[b] = r.prod[b].second; }
            long best = -1;
            std::array<int, NSLOT> bs{}, bn{};
            for (int pr = 0; pr < nperm(r.reac.size()); ++pr)
                for (int pp = 0; pp < nperm(r.prod.size()); ++pp) {
                    std::array<int, NSLOT> sa, na;
                    for (int q = 0; q < 3; ++q) {
                        sa[perms[pr][q]] = rs[q]; na[perms[pr][q]] = rn[q];
                        sa[3 + perms[pp][q]] = ps[q]; na[3 + perms[pp][q]] = pn[q];
                    }
                    long c = 0;
                    auto use = [&](long key) { auto it = cnt.find(key); if (it != cnt.end()) c += it->second; };
                    for (int a = 0; a < NSLOT; ++a) {
                        if (!na[a]) continue;
                        use(code(0, a, sa[a]));
                        if (sa[a] == bath) continue;
                        use(code(1, a, sa[a]));
                        for (int b = 0; b < NSLOT; ++b)
                            if (na[b] && (b < 3 || r.rev)) use(code(2, a * NSLOT + b, (long)sa[a] * 65536 + sa[b]));
                    }
                    if (best < 0 || c < best) { best = c; bs = sa; bn = na; }
                }
            for (int a = 0; a < NSLOT; ++a) {
                if (!bn[a]) continue;
                cnt[code(0, a, bs[a])]++;
                if (bs[a] == bath) continue;
                cnt[code(1, a, bs[a])]++;
                for (int b = 0; b < NSLOT; ++b)
                    if (bn[b] && (b < 3 || r.rev)) cnt[code(2, a * NSLOT + b, (long)bs[a] * 65536 + bs[b])]++;
            }
            SPA[p] = bs;
            NUA[p] = bn;
        }
    }

    for (int p = 0; p < nr_pad; ++p) {
        RxnRec& R = rec[p];
        for (int a = 0; a < NSLOT; ++a) R.sp[a] = (uint16_t)ns;
        R.eff = 0;
        R.neff = 0;
        if (p >= nr) continue;
        const auto& r = m.rx[m.order[p]];
        int spa[NSLOT], nua[NSLOT];
        for (int a = 0; a < NSLOT; ++a) { spa[a] = SPA[p][a]; nua[a] = NUA[p][a]; }
        bool bathdep = depends_on_bath(m, r);
        uint32_t w = 0;
        for (int a = 0; a < NSLOT; ++a) w |= (uint32_t)nua[a] << (4 * a);
        w |= (uint32_t)r.kind << 24;
        if (r.rev) w |= INFO_REV;
        if (bathdep) w |= INFO_BATH;
        for (int a = 0; a < NSLOT; ++a)
            if (nua[a] && spa[a] == bath) w |= INFO_BATHROW;
        R.info = w;
        double sumnu = 0, om = 0;
        for (int a = 0; a < NSLOT; ++a) {
            R.sp[a] = (uint16_t)spa[a];
            if (!nua[a]) continue;
            double nu = a < 3 ? -nua[a] : nua[a];
            sumnu += nu;
            om += nu * wfac[spa[a]];
        }
        R.dnu = sumnu;
        R.domega = om;
        R.lnA = r.lnA;
        R.b = r.b;
        R.theta = r.theta;
        if (r.chemact) R.info |= INFO_CHEMACT;
        if (kind_falloff(r.kind)) {
            fall[p].lnA0 = r.lnA0;
            fall[p].b0 = r.b0;
            fall[p].theta0 = r.theta0;
        }
        if (r.kind == K_TROE) {
            fall[p].p[0] = r.alpha;
            fall[p].p[1] = 1.0 / r.T3;
            fall[p].p[2] = 1.0 / r.T1;
            fall[p].p[3] = r.T2;
        }
        if (r.kind == K_SRI) {
            fall[p].p[0] = r.sri[0];
            fall[p].p[1] = r.sri[1];
            fall[p].p[2] = 1.0 / r.sri[2];
            fall[p].p[3] = std::log10(r.sri[3]);
            fall[p].p[4] = r.sri[4];
        }
        if (kind_table(r.kind)) {
            if (tabs.size() >= 65535) { err = "more than 65535 reactions tabulated in pressure"; return PJ_E_UNSUPPORTED; }
            TabRec tr{};
            tr.off = (int32_t)tabd.size();
            if (r.kind == K_PLOG) {
                tr.n = (int32_t)r.plog.size();
                for (const auto& pt : r.plog) {
                    const double row[PLOG_STRIDE] = {pt[0], std::log(pt[0]), pt[1], pt[2], pt[3], 0.0};
                    tabd.insert(tabd.end(), row, row + PLOG_STRIDE);
                }
            } else {
                // Tr = (2/T - 1/Tmin - 1/Tmax) / (1/Tmax - 1/Tmin) = ta / T + tb,
                // Pr = (2 ln P - ln Pmin - ln Pmax) / (ln Pmax - ln Pmin) = pa ln P + pb
                const double iT0 = 1.0 / r.cheb_T[0], iT1 = 1.0 / r.cheb_T[1];
                const double l0 = std::log(r.cheb_P[0]), l1 = std::log(r.cheb_P[1]);
                tr.n = r.cheb_nt;
                tr.np = r.cheb_np;
                tr.ta = 2.0 / (iT1 - iT0);
                tr.tb = -(iT0 + iT1) / (iT1 - iT0);
                tr.pa = 2.0 / (l1 - l0);
                tr.pb = -(l0 + l1) / (l1 - l0);
                for (double a : r.cheb) tabd.push_back(LN10 * a);
            }
            R.tab = (uint16_t)tabs.size();
            tabs.push_back(tr);
        }
        // rows: species of the reaction other than the bath gas
        JacRec& Jr = jrec[p];
        for (int a = 0; a < NSLOT; ++a) {
            if (!nua[a] || spa[a] == bath) continue;
            Jr.rowbase[a] = (uint16_t)m.row_ptr[2 + spa[a]];
            if (bathdep && !(m.opts & PJ_OPT_APPROX_JACOBIAN)) dense_row[spa[a]] = 1;
            for (int b = 0; b < NSLOT; ++b) {
                bool dep = nua[b] && (b < 3 || r.rev) && spa[b] != bath;
                if (!dep) continue;
                int sl = csr_find(m, 2 + spa[a], 2 + spa[b]);
                if (sl < 0) { err = "internal: pattern misses a reaction entry"; return PJ_E_UNSUPPORTED; }
                Jr.slot[a * NSLOT + b] = (uint16_t)sl;
            }
        }
        if (r.kind == K_THREEBODY || kind_falloff(r.kind)) {
            EffRec E;
            empty_eff(E);
            int ne = 0;
            for (auto& e : enhanced(r)) {
                E.sp[ne] = (uint16_t)e.first;
                E.am1[ne] = e.second - 1.0;
                if (e.first == bath) R.bam1 = e.second - 1.0;
                for (int a = 0; a < NSLOT; ++a) {
                    if (nua[a] && spa[a] != bath && e.first != bath) {
                        int f = csr_find(m, 2 + spa[a], 2 + e.first);
                        if (f < 0) { err = "internal: pattern misses a third-body entry"; return PJ_E_UNSUPPORTED; }
                        E.slot[a][ne] = (uint16_t)f;
                    }
                }
                ++ne;
            }
            R.eff = (uint32_t)effrec.size();
            R.neff = (uint32_t)ne;
            effrec.push_back(E);
        }
    }
    // per 64-reaction chunk: which slot positions any of its reactions uses
    // (bits 0..5), whether any is reversible (bit 6), the largest number of
    // third bodies of its reactions (bits 8..11), and which of the further
    // reaction types occur in it (bits 12..14); copied into every record
    std::vector<uint32_t> chunk((size_t)nr_pad / 64, 0);
    for (int p = 0; p < nr; ++p) {
        uint32_t& cm = chunk[p / 64];
        for (int a = 0; a < NSLOT; ++a) if (NUA[p][a]) cm |= 1u << a;
        if (rec[p].info & INFO_REV) cm |= 1u << 6;
        const int kd = info_kind(rec[p].info);
        if (kind_table(kd)) cm |= CHUNK_TAB;
        if (kd == K_SRI) cm |= CHUNK_SRI;
        if (rec[p].info & INFO_CHEMACT) cm |= CHUNK_CHEMACT;
        const uint32_t ne = std::max((cm >> 8) & 0xFu, rec[p].neff);
        cm = (cm & ~(0xFu << 8)) | (ne << 8);
    }
    for (int p = 0; p < nr_pad; ++p) rec[p].chunk = chunk[p / 64];
    std::vector<int32_t> dense_rows;
    for (int k = 0; k < ns; ++k) if (dense_row[k]) dense_rows.push_back(k);
    std::vector<uint16_t> col16(m.col_idx.begin(), m.col_idx.end());
    std::vector<uint16_t> row16(m.nnz);
    for (int i = 0; i < N; ++i)
        for (int e = m.row_ptr[i]; e < m.row_ptr[i + 1]; ++e) row16[e] = (uint16_t)i;
    std::vector<int32_t> orig(m.order.begin(), m.order.end());
    // CSR position -> column-order position
    std::vector<uint16_t> ccs(m.nnz);
    {
        std::vector<int32_t> next(m.col_ptr.begin(), m.col_ptr.end() - 1);
        for (int i = 0; i < N; ++i)
            for (int e = m.row_ptr[i]; e < m.row_ptr[i + 1]; ++e) ccs[e] = (uint16_t)next[m.col_idx[e]]++;
    }
    const int n_dense = (int)dense_rows.size();
    if (dense_rows.empty()) dense_rows.push_back(-1);
    if (tabs.empty()) tabs.push_back(TabRec{});
    if (tabd.empty()) tabd.push_back(0.0);

    // ---- one device buffer
    size_t total = 0;
    auto place = [&](size_t bytes) { size_t o = (total + 255) / 256 * 256; total = o + bytes; return o; };
    size_t o_th = place(th.size() * sizeof(ThermoRec)), o_tmid = place(tmid.size() * 8),
           o_wfac = place(wfac.size() * 8);
    size_t o_rec = place(rec.size() * sizeof(RxnRec)), o_fall = place(fall.size() * sizeof(FallRec)),
           o_jrec = place(jrec.size() * sizeof(JacRec));
    size_t o_eff = place(effrec.size() * sizeof(EffRec));
    size_t o_tab = place(tabs.size() * sizeof(TabRec)), o_tabd = place(tabd.size() * 8);
    size_t o_rowp = place(m.row_ptr.size() * 4), o_col = place(col16.size() * 2),
           o_dr = place(dense_rows.size() * 4);
    // dense maps: CSR slot of every (row, column), row-major and column-major
    std::vector<uint16_t> dmrm((size_t)N * N, NOSLOT), dmcm((size_t)N * N, NOSLOT);
    for (int i = 0; i < N; ++i)
        for (int e = m.row_ptr[i]; e < m.row_ptr[i + 1]; ++e) {
            dmrm[(size_t)i * N + m.col_idx[e]] = (uint16_t)e;
            dmcm[(size_t)i + (size_t)N * m.col_idx[e]] = (uint16_t)e;
        }
    for (int j = 0; j < N; ++j) dmcm[(size_t)N * j] = dmcm[1 + (size_t)N * j] = DMAP_SKIP;
    size_t o_rowof = place(row16.size() * 2), o_orig = place(orig.size() * 4), o_ccs = place(ccs.size() * 2);
    size_t o_dmrm = place(dmrm.size() * 2), o_dmcm = place(dmcm.size() * 2);
    std::vector<unsigned char> host(total, 0);
    auto put = [&](size_t off, const void* src, size_t bytes) { std::memcpy(host.data() + off, src, bytes); };
    put(o_th, th.data(), th.size() * sizeof(ThermoRec));
    put(o_tmid, tmid.data(), tmid.size() * 8);
    put(o_wfac, wfac.data(), wfac.size() * 8);
    put(o_rec, rec.data(), rec.size() * sizeof(RxnRec));
    put(o_fall, fall.data(), fall.size() * sizeof(FallRec));
    put(o_jrec, jrec.data(), jrec.size() * sizeof(JacRec));
    put(o_eff, effrec.data(), effrec.size() * sizeof(EffRec));
    put(o_tab, tabs.data(), tabs.size() * sizeof(TabRec));
    put(o_tabd, tabd.data(), tabd.size() * 8);
    put(o_rowp, m.row_ptr.data(), m.row_ptr.size() * 4);
    put(o_col, col16.data(), col16.size() * 2);
    put(o_dr, dense_rows.data(), dense_rows.size() * 4);
    put(o_rowof, row16.data(), row16.size() * 2);
    put(o_orig, orig.data(), orig.size() * 4);
    put(o_ccs, ccs.data(), ccs.size() * 2);
    put(o_dmrm, dmrm.data(), dmrm.size() * 2);
    put(o_dmcm, dmcm.data(), dmcm.size() * 2);

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { err = "no HIP device"; return PJ_E_DEVICE; }
    void* d = nullptr;
    if (hipMalloc(&d, total) != hipSuccess) { err = "hipMalloc of the mechanism tables failed"; return PJ_E_DEVICE; }
    if (hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        err = "copy of the mechanism tables failed";
        return PJ_E_DEVICE;
    }
    m.device = dev;
    m.dbuf = d;
    auto P = [&](size_t off) { return (const void*)((const unsigned char*)d + off); };
    DevMech& dm = m.dm;
    dm.ns = ns;
    dm.nr = nr;
    dm.nr_pad = nr_pad;
    dm.N = N;
    dm.nnz = m.nnz;
    dm.n_dense_rows = n_dense;
    dm.bath = bath;
    dm.th = gptr((const ThermoRec*)P(o_th));
    dm.tmid = gptr((const double*)P(o_tmid));
    dm.wfac = gptr((const double*)P(o_wfac));
    dm.rec = gptr((const RxnRec*)P(o_rec));
    dm.fall = gptr((const FallRec*)P(o_fall));
    dm.jrec = gptr((const JacRec*)P(o_jrec));
    dm.effrec = gptr((const EffRec*)P(o_eff));
    dm.tab = gptr((const TabRec*)P(o_tab));
    dm.tabd = gptr((const double*)P(o_tabd));
    dm.row_ptr = gptr((const int32_t*)P(o_rowp));
    dm.col_idx = gptr((const uint16_t*)P(o_col));
    dm.dense_rows = gptr((const int32_t*)P(o_dr));
    dm.row_of = gptr((const uint16_t*)P(o_rowof));
    dm.orig = gptr((const int32_t*)P(o_orig));
    dm.ccs_pos = (m.opts & PJ_OPT_CCS) ? gptr((const uint16_t*)P(o_ccs)) : nullptr;
    dm.dmap_rm = gptr((const uint16_t*)P(o_dmrm));
    dm.dmap_cm = gptr((const uint16_t*)P(o_dmcm));
    dm.arr = nullptr;
    dm.approx = (m.opts & PJ_OPT_APPROX_JACOBIAN) ? 1 : 0;
    dm.lsearch = (m.opts & PJ_OPT_LINEAR_SEARCH) ? 1 : 0;
    dm.det = (m.opts & PJ_OPT_DETERMINISTIC) ? 1 : 0;
    dm.ext = 0;
    for (const auto& r : m.rx)
        if (r.kind == K_SRI || r.chemact || kind_table(r.kind)) dm.ext = 1;
    m.h_rec = rec;
    m.off_rec = o_rec;

    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 65536;
    m.lds_max = lds_max;
    if (lds_bytes(dm, MODE_SRC, 1, 1) > lds_max) {
        err = "source-term working set exceeds the LDS of one workgroup";
        return PJ_E_UNSUPPORTED;
    }
    choose_launch(m);
    return PJ_OK;
}

}  // namespace pj
