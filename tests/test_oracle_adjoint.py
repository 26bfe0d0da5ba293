"""Pins of the oracle's adjoint: J^T v and the derivatives of v . dPhi/dt
with respect to every reaction's Arrhenius parameters (ln A, b, Ea/R; the
high-pressure limit's for falloff reactions), summed over the states.

Checked against facts other than the oracle's own chain rule: the closed form
for a one-reaction mechanism (dPhi/dt is proportional to k_f, so the
ln A-derivative equals v . dPhi/dt), complex-step derivatives in the
parameters, central differences of rewritten descriptions, and the duality
u . (J^T v) = v . (J u) with J u from a complex step in the state.
"""
import copy
import math

import numpy as np
import pytest

import oracle
from oracle.gates import WIDEN
from paper_1809_01029_amd import synth
from conftest import TINY_SEEDS, tiny_file, workload_file
from test_oracle_pins import _abc, _abc_state, write


def _states(m, n, seed, form):
    st = synth.make_states(m, n, seed)
    return synth.pack_state(st, form, "C")


def _v(n, N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, N))


@pytest.mark.parametrize("rtype,rev", [("ELEM", True), ("ELEM", False), ("THREEBODY", True)])
@pytest.mark.parametrize("form", ["conp", "conv"])
def test_param_grad_one_reaction_closed_form(tmp_path, rtype, rev, form):
    # one reaction: every source term is proportional to q = c R, and R to k_f,
    # so d(v.f)/d ln A = v.f, d/db = ln T v.f, d/d(Ea/R) = -v.f / T
    eff = [(0, 2.5), (2, 0.6)] if rtype == "THREEBODY" else ()
    m, o = _abc(tmp_path, rtype=rtype, rev=rev, eff=eff)
    xs, ps = [], []
    for T, nA in [(900.0, 0.02), (1300.0, 0.01), (2000.0, 0.05)]:
        x, P = _abc_state(T=T, nA=nA)
        if form == "conv":
            x = x.copy()
            x[1], P = P, x[1]
        xs.append(x)
        ps.append(P)
    x, p = np.array(xs), np.array(ps)
    v = _v(3, o.N, 5)
    f = o.source(x, p, form)
    vf = np.sum(v * f, axis=1)
    _, g = o.adjoint(x, p, v, form)
    T = x[:, 0]
    np.testing.assert_allclose(g[0, 0], vf.sum(), rtol=1e-12)
    np.testing.assert_allclose(g[1, 0], (vf * np.log(T)).sum(), rtol=1e-12)
    np.testing.assert_allclose(g[2, 0], -(vf / T).sum(), rtol=1e-12)


def test_param_grad_falloff_differs_from_proportional_form(tmp_path):
    # a falloff rate is not proportional to k_inf (c depends on Pr = k0 [M] / k_inf):
    # the derivative must carry the extra -(Rf - Rr) Pr dc/dPr term, which the
    # complex step confirms
    m, o = _abc(tmp_path, rtype="LINDEMANN", low=(40.0, -0.5, 2000.0))
    x, P = _abc_state()
    x, p = x[None, :], np.array([P])
    v = _v(1, o.N, 9)
    _, g = o.adjoint(x, p, v)
    vf = float(np.sum(v * o.source(x, p)))
    gcs = o.param_grad_cs(x, p, v)
    np.testing.assert_allclose(g, gcs, rtol=1e-11)
    assert abs(g[0, 0] - vf) > 1e-3 * abs(vf)


@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TINY_SEEDS)
@pytest.mark.parametrize("bath", [False, True])
def test_param_grad_matches_complex_step(form, seed, bath, mech_dir):
    kw = dict(bath_reactions=1, bath_efficiency=True) if bath else {}
    m, path = tiny_file(seed, mech_dir, **kw)
    o = oracle.Oracle(path)
    x, p = _states(m, 5, 40 + seed, form)
    v = _v(5, o.N, seed)
    _, g, _, gb = o.adjoint(x, p, v, form, bound=True)
    gcs = o.param_grad_cs(x, p, v, form)
    err = np.abs(g - gcs)
    allow = 1e-11 * np.abs(g) + WIDEN * gb + 1e-300
    assert np.all(err <= allow), float(np.max(err / allow))


def test_param_grad_matches_central_differences(mech_dir):
    # rewrite the description with one parameter moved by +-h and difference
    m, path = workload_file("ns13", mech_dir)
    o = oracle.Oracle(path)
    x, p = _states(m, 4, 123, "conp")
    v = _v(4, o.N, 3)
    _, g = o.adjoint(x, p, v)
    rng = np.random.default_rng(17)
    picks = [(int(i), int(a)) for i, a in zip(rng.choice(len(m.reactions), 10), rng.integers(0, 3, 10))]
    for i, a in picks:
        r = m.reactions[i]
        base = (r.lnA, r.b, r.theta)[a]
        h = 1e-6 * max(abs(base), 1.0)
        vals = []
        for sgn in (1, -1):
            m2 = copy.deepcopy(m)
            r2 = m2.reactions[i]
            if a == 0:
                r2.lnA = base + sgn * h
            elif a == 1:
                r2.b = base + sgn * h
            else:
                r2.theta = base + sgn * h
            p2 = path + f".fd_{i}_{a}_{sgn}.pjm"
            synth.write_mechanism(m2, p2)
            vals.append(float(np.sum(v * oracle.Oracle(p2).source(x, p))))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert fd == pytest.approx(g[a, i], rel=2e-5, abs=1e-9 * abs(g).max()), (i, a)


@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("name,n", [("tiny", 6), ("ns13", 6), ("ns53", 2)])
def test_jtv_duality_with_complex_step(form, name, n, mech_dir):
    if name == "tiny":
        m, path = tiny_file(11, mech_dir, bath_reactions=1, bath_efficiency=True)
    else:
        m, path = workload_file(name, mech_dir)
    o = oracle.Oracle(path)
    x, p = _states(m, n, 7, form)
    v = _v(n, o.N, 1)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(x.shape) * np.abs(x)        # directions on the state's scale
    jtv, _, jb, _ = o.adjoint(x, p, v, form, bound=True)
    ju = o.jvp_cs(x, p, u, form)
    lhs = np.sum(u * jtv, axis=1)
    rhs = np.sum(v * ju, axis=1)
    allow = np.sum(np.abs(u) * (1e-11 * np.abs(jtv) + WIDEN * jb), axis=1)
    assert np.all(np.abs(lhs - rhs) <= allow), np.max(np.abs(lhs - rhs) / allow)
