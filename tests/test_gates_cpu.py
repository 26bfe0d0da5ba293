"""The paper's error norms as written in oracle.gates (Sec. 3.2 E_X; Sec. 3.3
E_C and E_L), pinned by values worked out by hand."""
import math

import numpy as np

from oracle import gates


def test_e_x_weights():
    # |ref - g| / (1e-10 + 1e-6 |ref|): 1e-10 / (1e-10 + 1e-10) = 0.5
    assert math.isclose(gates.e_x(np.array([1e-4 + 1e-10]), np.array([1e-4])), 0.5, rel_tol=1e-6)
    # the largest over the entries; a zero reference weighs by 1e-10 alone
    assert math.isclose(gates.e_x(np.array([3e-10, 1.0]), np.array([0.0, 1.0])), 3.0, rel_tol=1e-12)


def test_e_l_uniform_relative_error():
    rng = np.random.default_rng(1)
    J = rng.standard_normal((5, 4, 4))
    assert gates.e_l(J, J) == 0.0
    # every state off by the same relative 1e-9: 1e-9 per state, sqrt(5) 1e-9 over 5 states
    assert math.isclose(gates.e_l(J * (1 + 1e-9), J), math.sqrt(5) * 1e-9, rel_tol=1e-6)


def test_e_c_filter():
    # two states, one large and one small entry each; T = Frobenius norm of all
    J = np.zeros((2, 2, 2))
    J[:, 0, 0] = 1.0
    J[:, 1, 1] = 1e-12
    T = math.sqrt(2 * (1.0 + 1e-24))
    G = J * (1 + 1e-6)
    # C = 1e6: T / C ~ 1.4e-6 keeps only the two 1.0 entries: sqrt(2) 1e-6
    assert math.isclose(gates.e_c(G, J, 1e6), math.sqrt(2) * 1e-6, rel_tol=1e-6)
    # C = 1e20 keeps all four entries: sqrt(4) 1e-6
    assert T / 1e20 < 1e-12
    assert math.isclose(gates.e_c(G, J, 1e20), 2e-6, rel_tol=1e-6)


def test_literal_report_counts():
    ref = np.array([1.0, 1.0, 2.0, 0.0])
    b = np.array([1e-16, 1e-16, 1e-16, 0.0])
    g = np.array([1.0 + 2e-10, 1.0, 2.0 - 1e-11, 0.0])
    r = gates.literal_report(g, ref, b, 1e-10)
    assert r["n_entries"] == 4 and r["n_literal_fail"] == 1
    assert math.isclose(r["max_rel_err"], 2e-10, rel_tol=1e-5)
    # kappa = b / (u |ref|) of the failing entry
    assert math.isclose(r["literal_fail_kappa"][0], 1e-16 / (2.0 ** -53), rel_tol=1e-12)
