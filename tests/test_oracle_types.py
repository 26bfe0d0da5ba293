"""Pins of the oracle's further reaction types: SRI falloff, chemically
activated reactions (Lindemann, Troe and SRI forms), pressure-dependent
Arrhenius (P-Log) and Chebyshev rate constants.

The paper names these types as supported without restating their formulas;
the oracle takes the standard definitions (SRI: F = d (a e^(-b/T) +
e^(-T/c))^X T^e with X = 1/(1 + log10(Pr)^2); chemically activated:
c = F/(1 + Pr) on a rate with the low-pressure limit; P-Log: ln k linear in
ln P between tabulated pressures; Chebyshev: log10 k a double Chebyshev series
in reduced 1/T and log P).  These tests check it against closed forms written
out here, the textbook special cases (SRI with F = 1 is Lindemann, a one-point
P-Log is an Arrhenius rate), numpy's own Chebyshev series, conservation laws,
a constructed equilibrium, and complex-step and central-difference derivatives
for the Jacobian and the adjoint.
"""
import copy
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle
from paper_1809_01029_amd import synth
from conftest import TYPES_SEEDS, types_file, workload_file
from oracle.gates import WIDEN
from test_oracle_pins import SPECIES_ABC, _check_cs, fd_allowance, micro, state_vec, write

R = 8314.462618
PREF = 101325.0
ATM = 101325.0


def _rx(rtype, lnA=30.0, b=0.7, th=5000.0, **kw):
    return synth.Reaction(rtype, True, [(0, 1), (1, 1)], [(2, 1)], lnA, b, th, **kw)


def _one(tmp_path, rx, name):
    m = micro(SPECIES_ABC, [rx])
    return m, write(m, tmp_path, name)


def _arr(lnA, b, th, T):
    return math.exp(lnA + b * math.log(T) - th / T)


def _x(T, P, V=1.0, fr=(0.2, 0.15, 0.3)):
    ntot = P * V / (R * T)
    return state_vec(T, V, [f * ntot for f in fr])


LOW = (40.0, -0.5, 2000.0)
SRI = (0.8, 600.0, 900.0, 1.3, 0.2)
TROE = (0.35, 800.0, 2500.0, 4000.0)


# ---------------------------------------------------------------------------
# SRI falloff

@pytest.mark.parametrize("eff", [(), ((0, 2.5), (2, 0.6))])
def test_sri_closed_form(tmp_path, eff):
    m, o = _one(tmp_path, _rx("SRI", low=LOW, sri=SRI, eff=list(eff)), f"sri{len(eff)}")
    for T, P in [(900.0, 2 * ATM), (1300.0, 3 * ATM), (2100.0, 40 * ATM)]:
        x = _x(T, P)
        c = o.components(x, P)
        C = c["C"]
        M = P / (R * T) + sum((a - 1.0) * C[s] for s, a in eff)
        kinf = _arr(30.0, 0.7, 5000.0, T)
        k0 = _arr(*LOW, T)
        Pr = k0 * M / kinf
        a, b, cc, d, e = SRI
        X = 1.0 / (1.0 + math.log10(Pr) ** 2)
        F = d * (a * math.exp(-b / T) + math.exp(-T / cc)) ** X * T ** e
        assert c["kf"][0] == pytest.approx(kinf, rel=1e-13)
        assert c["c"][0] == pytest.approx(F * Pr / (1.0 + Pr), rel=1e-12)


def test_sri_with_unit_f_is_lindemann(tmp_path):
    # a = 0, c -> infinity, d = 1, e = 0: the SRI base is exp(-T/c) = 1, F = 1
    _, o1 = _one(tmp_path, _rx("SRI", low=LOW, sri=(0.0, 500.0, 1e300, 1.0, 0.0)), "sri_unit")
    _, o2 = _one(tmp_path, _rx("LINDEMANN", low=LOW), "lind_ref")
    for form in ("conp", "conv"):
        for T, P in [(900.0, 2 * ATM), (1700.0, 30 * ATM)]:
            x = _x(T, P)
            p = P
            if form == "conv":
                x = x.copy()
                x[1], p = P, x[1]
            f1, f2 = o1.source(x[None], np.array([p]), form), o2.source(x[None], np.array([p]), form)
            np.testing.assert_allclose(f1, f2, rtol=1e-14, atol=0)
            J1, J2 = o1.jacobian(x[None], np.array([p]), form), o2.jacobian(x[None], np.array([p]), form)
            np.testing.assert_allclose(J1, J2, rtol=1e-13, atol=1e-300)


# ---------------------------------------------------------------------------
# chemically activated reactions

def test_chemically_activated_lindemann_closed_form_and_limits(tmp_path):
    _, o = _one(tmp_path, _rx("LINDEMANN", low=LOW, chemact=True), "ca_lind")
    for T, P in [(1000.0, 1 * ATM), (1500.0, 20 * ATM)]:
        x = _x(T, P)
        c = o.components(x, P)
        k0, kinf = _arr(*LOW, T), _arr(30.0, 0.7, 5000.0, T)
        Pr = k0 * (P / (R * T)) / kinf
        # the rate constant is k0 F / (1 + Pr), F = 1
        assert c["kf"][0] == pytest.approx(k0, rel=1e-13)
        assert c["c"][0] == pytest.approx(1.0 / (1.0 + Pr), rel=1e-13)
    # Pr -> 0: the rate constant tends to k0; Pr -> infinity: to k_inf / [M]
    T = 1300.0
    k0, kinf = _arr(*LOW, T), _arr(30.0, 0.7, 5000.0, T)
    for P, lim in ((1e-12 * ATM, "lo"), (1e12 * ATM, "hi")):
        c = o.components(_x(T, P), P)
        M = P / (R * T)
        Pr = k0 * M / kinf
        keff = c["kf"][0] * c["c"][0]
        if lim == "lo":
            assert Pr < 1e-8 and keff == pytest.approx(k0, rel=10 * Pr + 1e-13)
        else:
            assert Pr > 1e8 and keff == pytest.approx(kinf / M, rel=10 / Pr + 1e-13)


@pytest.mark.parametrize("rtype,extra", [("TROE", {"troe": TROE}), ("SRI", {"sri": SRI})])
def test_chemically_activated_shares_the_falloff_broadening(tmp_path, rtype, extra):
    # same F(Pr, T) as the falloff form: c_falloff = F Pr/(1+Pr), c_chemact = F/(1+Pr)
    _, of = _one(tmp_path, _rx(rtype, low=LOW, **extra), f"fo_{rtype}")
    _, oc = _one(tmp_path, _rx(rtype, low=LOW, chemact=True, **extra), f"ca_{rtype}")
    for T, P in [(900.0, 2 * ATM), (1300.0, 3 * ATM), (2100.0, 40 * ATM)]:
        x = _x(T, P)
        cf, cc = of.components(x, P), oc.components(x, P)
        Pr = _arr(*LOW, T) * (P / (R * T)) / _arr(30.0, 0.7, 5000.0, T)
        assert cf["c"][0] / cc["c"][0] == pytest.approx(Pr, rel=1e-12)
        assert cc["kf"][0] == pytest.approx(_arr(*LOW, T), rel=1e-13)


# ---------------------------------------------------------------------------
# P-Log

PLOG = [(0.1 * ATM, 28.0, 0.5, 4000.0), (1.0 * ATM, 30.0, 0.2, 5000.0), (10.0 * ATM, 31.0, -0.3, 6000.0)]


def _lnk(pt, T):
    return pt[1] + pt[2] * math.log(T) - pt[3] / T


def test_plog_closed_forms(tmp_path):
    _, o = _one(tmp_path, _rx("PLOG", 0.0, 0.0, 0.0, plog=PLOG), "plog")
    T = 1300.0
    kf = lambda P: o.components(_x(T, P), P)["kf"][0]  # noqa: E731
    # at a tabulated pressure: that pressure's Arrhenius expression
    for pt in PLOG:
        assert kf(pt[0]) == pytest.approx(math.exp(_lnk(pt, T)), rel=1e-13)
    # between two: linear in ln P
    for P, (lo, hi) in [(3 * ATM, (1, 2)), (0.2 * ATM, (0, 1))]:
        a, b = PLOG[lo], PLOG[hi]
        w = (math.log(P) - math.log(a[0])) / (math.log(b[0]) - math.log(a[0]))
        assert kf(P) == pytest.approx(math.exp(_lnk(a, T) + w * (_lnk(b, T) - _lnk(a, T))), rel=1e-12)
    # outside the table: the nearest end
    assert kf(0.01 * ATM) == pytest.approx(math.exp(_lnk(PLOG[0], T)), rel=1e-13)
    assert kf(100 * ATM) == pytest.approx(math.exp(_lnk(PLOG[-1], T)), rel=1e-13)
    # the main Arrhenius expression multiplies the tabulated rate
    _, o2 = _one(tmp_path, _rx("PLOG", 0.3, 0.1, 200.0, plog=PLOG), "plog_f")
    P = 3 * ATM
    assert o2.components(_x(T, P), P)["kf"][0] == pytest.approx(kf(P) * _arr(0.3, 0.1, 200.0, T), rel=1e-12)


def test_one_point_plog_is_arrhenius(tmp_path):
    _, o1 = _one(tmp_path, _rx("PLOG", 0.0, 0.0, 0.0, plog=[(2 * ATM, 30.0, 0.7, 5000.0)]), "plog1")
    _, o2 = _one(tmp_path, _rx("ELEM"), "elem_ref")
    for form in ("conp", "conv"):
        for T, P in [(900.0, 0.5 * ATM), (1700.0, 30 * ATM)]:
            x = _x(T, P)
            p = P
            if form == "conv":
                x = x.copy()
                x[1], p = P, x[1]
            xa, pa = x[None], np.array([p])
            np.testing.assert_allclose(o1.source(xa, pa, form), o2.source(xa, pa, form), rtol=1e-13, atol=0)
            np.testing.assert_allclose(o1.jacobian(xa, pa, form), o2.jacobian(xa, pa, form),
                                       rtol=1e-12, atol=1e-300)


# ---------------------------------------------------------------------------
# Chebyshev

def _cheb_rx(coef, lnA=0.0, b=0.0, th=0.0):
    return _rx("CHEB", lnA, b, th, cheb=((300.0, 2500.0, 0.01 * ATM, 100.0 * ATM),
                                         [list(map(float, row)) for row in coef]))


def test_chebyshev_matches_numpy_series(tmp_path):
    rng = np.random.default_rng(4)
    coef = rng.normal(0.0, 0.4, size=(5, 3))
    coef[0, 0] = 11.0
    _, o = _one(tmp_path, _cheb_rx(coef), "cheb")
    for T in (350.0, 1300.0, 2400.0, 2800.0):
        for P in (0.05 * ATM, 1 * ATM, 50 * ATM, 200 * ATM):
            Tr = (2 / T - 1 / 300.0 - 1 / 2500.0) / (1 / 2500.0 - 1 / 300.0)
            Pr = (2 * math.log10(P) - math.log10(0.01 * ATM) - math.log10(100 * ATM)) / \
                 (math.log10(100 * ATM) - math.log10(0.01 * ATM))
            ref = 10.0 ** npcheb.chebval2d(Tr, Pr, coef)
            assert o.components(_x(T, P), P)["kf"][0] == pytest.approx(ref, rel=1e-12), (T, P)
    # one coefficient: a constant rate; a factor from the main Arrhenius expression
    _, o1 = _one(tmp_path, _cheb_rx([[9.5]], 0.3, 0.1, 200.0), "cheb1")
    T, P = 1100.0, 4 * ATM
    assert o1.components(_x(T, P), P)["kf"][0] == pytest.approx(10 ** 9.5 * _arr(0.3, 0.1, 200.0, T),
                                                              rel=1e-13)


# ---------------------------------------------------------------------------
# whole mechanisms with every type

def _states(m, n, seed, form):
    st = synth.make_states(m, n, seed)
    return synth.pack_state(st, form, "C")


def test_types_mechanisms_hold_every_type(mech_dir):
    for seed in TYPES_SEEDS:
        m, _ = types_file(seed, mech_dir)
        kinds = {(r.type, r.chemact) for r in m.reactions}
        for k in [("SRI", False), ("PLOG", False), ("CHEB", False), ("TROE", False)]:
            assert k in kinds
        assert any(r.chemact for r in m.reactions)


@pytest.mark.parametrize("seed", TYPES_SEEDS)
def test_types_conservation(seed, mech_dir):
    m, path = types_file(seed, mech_dir, bath=True)
    o = oracle.Oracle(path)
    x, p = _states(m, 5, seed, "conp")
    nu = np.zeros((m.n_species, m.n_reactions))
    for i, r in enumerate(m.reactions):
        for sp, v in r.reac:
            nu[sp, i] -= v
        for sp, v in r.prod:
            nu[sp, i] += v
    for s in range(x.shape[0]):
        c = o.components(x[s], p[s])
        absw = np.abs(nu) @ np.abs(c["q"])
        for e in range(4):
            assert abs(m.comp[:, e] @ c["wdot"]) <= 1e-12 * (m.comp[:, e] @ absw) + 1e-300
        assert abs(m.W @ c["wdot"]) <= 1e-12 * (m.W @ absw) + 1e-300


@pytest.mark.parametrize("seed", TYPES_SEEDS)
def test_types_conp_and_conv_agree(seed, mech_dir):
    # the same physical state gives the same rates in either form
    m, path = types_file(seed, mech_dir)
    o = oracle.Oracle(path)
    st = synth.make_states(m, 4, seed)
    xa, pa = synth.pack_state(st, "conp", "C")
    xv, pv = synth.pack_state(st, "conv", "C")
    for s in range(4):
        a, b = o.components(xa[s], pa[s], "conp"), o.components(xv[s], pv[s], "conv")
        np.testing.assert_allclose(a["q"], b["q"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", TYPES_SEEDS)
def test_types_detailed_balance(seed, mech_dir, tmp_path):
    m, _ = types_file(seed, mech_dir)
    m = copy.deepcopy(m)
    for r in m.reactions:
        r.rev = True
    o = write(m, tmp_path, f"teq{seed}")
    rng = np.random.default_rng(seed)
    for T in (800.0, 1500.0, 2100.0):
        g = np.array([o.thermo(k, T)[1] - o.thermo(k, T)[2] for k in range(m.n_species)])
        lam = rng.uniform(-2, 2, size=4)
        lam[3] = (g[-1] + math.log(0.5)) / 2.0
        C = PREF / (R * T) * np.exp(-g + m.comp @ lam)
        P = C.sum() * R * T
        x = state_vec(T, 1.0, C[:-1])
        c = o.components(x, P)
        assert np.all(np.abs(c["q"]) <= 1e-10 * np.abs(c["c"]) * np.abs(c["Rf"]) + 1e-300)


@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TYPES_SEEDS)
@pytest.mark.parametrize("bath", [False, True])
def test_types_jacobian_matches_complex_step(form, seed, bath, mech_dir):
    m, path = types_file(seed, mech_dir, bath=bath)
    o = oracle.Oracle(path)
    x, p = _states(m, 5, 70 + seed, form)
    J, Js, Jc = _check_cs(o, x, p, form)
    P = o.pattern()
    assert not np.any((Jc != 0) & ~P[None])


@pytest.mark.parametrize("form", ["conp", "conv"])
def test_types_workload_jacobian_matches_complex_step(form, mech_dir):
    m, path = workload_file("ns111x", mech_dir)
    o = oracle.Oracle(path)
    w = synth.WORKLOADS["ns111x"]
    st = synth.make_states(m, 2, w.state_seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
    x, p = synth.pack_state(st, form, "C")
    J, Js, Jc = _check_cs(o, x, p, form)
    assert not np.any((Jc != 0) & ~o.pattern()[None])


@pytest.mark.parametrize("form", ["conp", "conv"])
def test_types_jacobian_matches_central_differences(form, mech_dir):
    m, path = types_file(TYPES_SEEDS[0], mech_dir)
    o = oracle.Oracle(path)
    x, p = _states(m, 4, 9, form)
    J, Jb = o.jacobian(x, p, form, bound=True)
    Jf = o.jacobian_fd(x, p, form, rel=1e-6)
    f, fb = o.source(x, p, form, bound=True)
    h = 1e-6 * np.maximum(np.abs(x), 1e-300)
    tol = fd_allowance(J, Jb, f, fb, h)
    assert np.all(np.abs(J - Jf) <= tol), float(np.max(np.abs(J - Jf) / tol))


@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TYPES_SEEDS)
def test_types_param_grad_matches_complex_step(form, seed, mech_dir):
    m, path = types_file(seed, mech_dir, bath=True)
    o = oracle.Oracle(path)
    x, p = _states(m, 5, 90 + seed, form)
    v = np.random.default_rng(seed).standard_normal((5, o.N))
    _, g, _, gb = o.adjoint(x, p, v, form, bound=True)
    gcs = o.param_grad_cs(x, p, v, form)
    allow = 1e-11 * np.abs(g) + WIDEN * gb + 1e-300
    assert np.all(np.abs(g - gcs) <= allow), float(np.max(np.abs(g - gcs) / allow))


@pytest.mark.parametrize("rx", [_rx("PLOG", 0.0, 0.0, 0.0, plog=PLOG),
                                _cheb_rx([[11.0, 0.2], [-1.0, 0.05], [0.1, -0.02]])],
                         ids=["plog", "cheb"])
def test_types_param_grad_one_reaction_closed_form(tmp_path, rx):
    # the main Arrhenius expression multiplies the tabulated rate, so with one
    # reaction d(v.f)/d ln A = v.f, d/db = ln T v.f, d/d(Ea/R) = -v.f/T
    m, o = _one(tmp_path, rx, f"pg_{rx.type}")
    x = np.array([_x(T, P) for T, P in [(900.0, 0.5 * ATM), (1300.0, 3 * ATM), (2000.0, 40 * ATM)]])
    p = np.array([0.5 * ATM, 3 * ATM, 40 * ATM])
    v = np.random.default_rng(2).standard_normal((3, o.N))
    vf = np.sum(v * o.source(x, p), axis=1)
    _, g = o.adjoint(x, p, v)
    T = x[:, 0]
    np.testing.assert_allclose(g[:, 0], [vf.sum(), (vf * np.log(T)).sum(), -(vf / T).sum()], rtol=1e-12)
