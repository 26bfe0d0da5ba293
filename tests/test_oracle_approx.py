"""Pins of the oracle's approximate Jacobian (Sec. 3.4): the bath gas's moles
held fixed against the other species' moles (its dependence on T and V or P
kept).

Checked against a complex step through a closure whose species sum drops its
imaginary part (so the perturbation of n_j does not reach n_Ns), against the
exact Jacobian in the columns the approximation does not touch, and for
pattern soundness; the density change is compared in direction with the
paper's table.
"""
import os

import numpy as np
import pytest

import oracle
from oracle.gates import WIDEN
from paper_1809_01029_amd import synth
from conftest import TINY_SEEDS, tiny_file, workload_file

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TINY_SEEDS)
def test_approx_matches_frozen_complex_step(form, seed, mech_dir):
    m, path = tiny_file(seed, mech_dir, bath_reactions=1, bath_efficiency=True)
    o = oracle.Oracle(path)
    st = synth.make_states(m, 4, 70 + seed)
    x, p = synth.pack_state(st, form, "C")
    J, b = o.jacobian(x, p, form, bound=True, approx=True)
    Jcs = o.jacobian_cs(x, p, form, approx=True)
    allow = 1e-12 * np.abs(J) + WIDEN * b + 1e-300
    assert np.all(np.abs(J - Jcs) <= allow), float(np.max(np.abs(J - Jcs) / allow))
    # the frozen closure really is a different function: the exact complex
    # step differs from it somewhere in the species columns
    Jex = o.jacobian_cs(x, p, form)
    assert np.any(np.abs(Jex[:, :, 2:] - Jcs[:, :, 2:]) > 1e-6 * np.abs(Jex[:, :, 2:]).max())


@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("name", ["ns13", "ns53"])
def test_approx_keeps_temperature_and_state_columns(form, name, mech_dir):
    m, path = workload_file(name, mech_dir)
    o = oracle.Oracle(path)
    st = synth.make_states(m, 3, 5)
    x, p = synth.pack_state(st, form, "C")
    Ja = o.jacobian(x, p, form, approx=True)
    Je = o.jacobian(x, p, form)
    np.testing.assert_array_equal(Ja[:, :, :2], Je[:, :, :2])
    # and it lies on its own pattern
    P = o.pattern(approx=True)
    assert np.all(Ja[:, ~P] == 0)
    assert np.all(o.jacobian_cs(x, p, form, approx=True)[:, ~P] == 0)


def test_approx_pattern_is_sparser_like_the_paper(mech_dir):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "approx_jacobian_density.txt"))
            if l.strip() and not l.startswith("#")]
    for name, pe, pa in rows:
        m, path = workload_file(name, mech_dir)
        o = oracle.Oracle(path)
        de, da = o.pattern().mean(), o.pattern(approx=True).mean()
        # the approximation only removes entries, as in every model of the table
        assert da <= de and float(pa) < float(pe)
        assert np.all(o.pattern(approx=True) <= o.pattern())


@pytest.mark.parametrize("seed", TINY_SEEDS)
def test_approx_pattern_is_exactly_the_support(seed, mech_dir):
    # with a bath gas that reacts and has a third-body efficiency other than
    # one, the species block of the approximate pattern is exactly the set of
    # entries the frozen-closure complex step finds non-zero (plus the diagonal)
    m, path = tiny_file(seed, mech_dir, bath_reactions=1, bath_efficiency=True)
    o = oracle.Oracle(path)
    st = synth.make_states(m, 3, 90 + seed)
    x, p = synth.pack_state(st, "conp", "C")
    nz = np.any(o.jacobian_cs(x, p, "conp", approx=True) != 0, axis=0)
    P = o.pattern(approx=True)
    N = o.N
    want = nz[2:, 2:] | np.eye(N - 2, dtype=bool)
    np.testing.assert_array_equal(P[2:, 2:], want)
