"""The seeded input generators: validity of what they build."""
import os

import numpy as np
import pytest

import oracle
ATM = 101325.0
from paper_1809_01029_amd import synth
from conftest import TINY_SEEDS, tiny_file, workload_file

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_deterministic_and_round_trip():
    a = synth.dumps(synth.make_mechanism(20, 40, 5))
    b = synth.dumps(synth.make_mechanism(20, 40, 5))
    assert a == b
    assert synth.dumps(synth.loads(a)) == a
    assert synth.dumps(synth.make_mechanism(20, 40, 6)) != a


@pytest.mark.parametrize("name", list(synth.WORKLOADS))
def test_workload_mechanism_valid(name, mech_dir):
    m, path = workload_file(name, mech_dir)
    w = synth.WORKLOADS[name]
    assert m.n_species == w.ns and m.n_reactions == w.nr
    bath = m.n_species - 1
    seen = set()
    counts = {"ELEM_REV": 0, "ELEM_IRR": 0, "THREEBODY": 0, "LINDEMANN": 0, "TROE": 0, "SRI": 0,
              "PLOG": 0, "CHEB": 0, "CHEMACT": 0}
    for r in m.reactions:
        lhs = sum(nu * m.comp[s] for s, nu in r.reac)
        rhs = sum(nu * m.comp[s] for s, nu in r.prod)
        assert np.array_equal(lhs, rhs), "element balance"
        assert sum(nu for _, nu in r.reac) <= 3 and sum(nu for _, nu in r.prod) <= 3
        assert all(nu in (1, 2) for _, nu in r.reac + r.prod)
        assert not ({s for s, _ in r.reac} & {s for s, _ in r.prod})
        key = (tuple(r.reac), tuple(r.prod))
        assert key not in seen and (key[1], key[0]) not in seen
        seen.add(key)
        kind = r.type if r.type != "ELEM" else ("ELEM_REV" if r.rev else "ELEM_IRR")
        counts["CHEMACT" if r.chemact else kind] += 1
        if r.type in ("PLOG", "CHEB"):
            # the main Arrhenius expression is a unit factor on the tabulated rate
            assert (r.lnA, r.b, r.theta) == (0.0, 0.0, 0.0) and not r.eff
        else:
            assert 8 * np.log(10) <= r.lnA <= 16 * np.log(10) and -2 <= r.b <= 3 and 0 <= r.theta <= 3e4
        if r.type == "PLOG":
            ps = [pt[0] for pt in r.plog]
            assert 2 <= len(ps) <= 5 and all(a < b for a, b in zip(ps, ps[1:]))
            assert 0.1 * ATM * 0.999 <= ps[0] and ps[-1] <= 10 ** 2.5 * ATM * 1.001
        if r.type == "CHEB":
            (tmin, tmax, pmin, pmax), coef = r.cheb
            assert tmin < 600 and tmax > 2200 and pmin < ATM and pmax > 60 * ATM
            assert 3 <= len(coef) <= 6 and 2 <= len(coef[0]) <= 4
        if r.type in ("THREEBODY",) + synth.FALLOFF_TYPES:
            assert 1 <= len(r.eff) <= 6 and all(0.5 <= a <= 5 for _, a in r.eff)
            assert all(s != bath for s, _ in r.eff)
        if r.type == "TROE":
            al, t3, t1, t2 = r.troe
            assert 0 <= al <= 1 and all(100 <= t <= 5000 for t in (t3, t1, t2))
    nr = w.nr
    assert counts["THREEBODY"] == round(w.mix.third_body * nr)
    assert counts["LINDEMANN"] + counts["TROE"] == round(w.mix.falloff * nr)
    assert abs(counts["LINDEMANN"] - counts["TROE"]) <= 1
    assert counts["ELEM_IRR"] == round(w.mix.irreversible * nr)
    assert counts["SRI"] == round(w.mix.sri * nr) and counts["CHEMACT"] == round(w.mix.chem_act * nr)
    assert counts["PLOG"] == round(w.mix.plog * nr) and counts["CHEB"] == round(w.mix.cheb * nr)
    # the bath gas takes part in exactly the requested number of reactions
    nb = sum(1 for r in m.reactions if bath in [s for s, _ in r.reac + r.prod])
    assert nb == w.bath_reactions


def test_densities_near_paper_table(mech_dir):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "jacobian_density.txt"))
            if l.strip() and not l.startswith("#")]
    for name, dens, dev in rows:
        m, path = workload_file(name, mech_dir)
        P = oracle.Oracle(path).pattern()
        got = P.sum() / P.size
        assert abs(got - float(dens)) <= float(dev), (name, got)


def test_states_distribution():
    m = synth.make_mechanism(20, 40, 5)
    st = synth.make_states(m, 5000, 9, T_range=(600, 2200), P_range_atm=(1, 50))
    assert st["T"].min() >= 600 and st["T"].max() <= 2200
    assert st["P"].min() >= synth.ATM and st["P"].max() <= 50 * synth.ATM
    assert np.all(st["n"] > 0)
    ntot = st["P"] * st["V"] / (synth.R_GAS * st["T"])
    np.testing.assert_allclose(st["n"].sum(axis=1), ntot, rtol=1e-13)
    xc, pc = synth.pack_state(st, "conp", "C")
    xf, pf = synth.pack_state(st, "conp", "F")
    assert xc.shape == (5000, 21) and xf.shape == (21, 5000)
    np.testing.assert_array_equal(xc.T, xf)
    np.testing.assert_array_equal(pc, st["P"])
    xv, pv = synth.pack_state(st, "conv", "C")
    np.testing.assert_array_equal(xv[:, 1], st["P"])
    np.testing.assert_array_equal(pv, st["V"])


@pytest.mark.parametrize("seed", TINY_SEEDS)
def test_tiny_mechanisms_have_every_type(seed, mech_dir):
    m, _ = tiny_file(seed, mech_dir, bath_reactions=1, bath_efficiency=True)
    types = {r.type for r in m.reactions}
    assert types == {"ELEM", "THREEBODY", "LINDEMANN", "TROE"}
    assert any(not r.rev for r in m.reactions)
    bath = m.n_species - 1
    assert any(bath in [s for s, _ in r.reac] for r in m.reactions)
    assert any(bath in [s for s, _ in r.eff] for r in m.reactions)
