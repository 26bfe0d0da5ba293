"""Parity gates of the HIP path against the oracle, and the paper's error norms.

The stated tolerances are relative: 1e-10 for source terms, 1e-8 (with an
absolute floor of 1e-20) for Jacobian entries, J^T v and parameter
gradients.  Where an entry cancels (near-equilibrium net rates, the paper's
Sec. 3.2 source-term error table) two correct FP64 evaluations can differ by
more than that relative amount, so the gate also uses the oracle's running
error bound b of the entry (a first-order bound on |oracle - exact|):

    allowed = tol |ref| + floor                 where b <= (tol / 100) |ref|
    allowed = tol |ref| + floor + WIDEN * b     otherwise

On a well-conditioned entry (the common case) this is the literal relative
test.  WIDEN covers the different order and grouping of the same operations
in another correct code; a pin checks that reordering the reactions of a
mechanism keeps the oracle inside its own gate.

The error norms follow Sec. 3.2 (E_X, Eq. of the relative error norm) and
Sec. 3.3 (the filtered E_C and the LAPACK-style E_L of the Jacobian).
"""
from __future__ import annotations

import numpy as np

SRC_TOL = 1e-10
JAC_TOL = 1e-8
JAC_ABS = 1e-20
WIDEN = 16.0
U_ROUND = 2.0 ** -53


def allowance(ref, bound, tol, floor=0.0):
    """Largest |value - ref| accepted for an entry the oracle evaluates as
    ``ref`` with running error bound ``bound``."""
    a = np.abs(ref)
    widened = bound > (tol / 100.0) * a
    return tol * a + floor + np.where(widened, WIDEN * bound, 0.0)


def src_allowance(ref, bound):
    return allowance(ref, bound, SRC_TOL)


def jac_allowance(ref, bound):
    return allowance(ref, bound, JAC_TOL, JAC_ABS)


def _check(g, ref, bound, tol, floor, what, kind):
    g = np.asarray(g)
    err = np.abs(g - ref)
    allow = allowance(ref, bound, tol, floor)
    bad = ~(err <= allow)
    if bad.any():
        worst = float(np.nanmax(np.where(np.isfinite(err), err / np.maximum(allow, 1e-300), np.inf)))
        i = np.unravel_index(int(np.argmax(np.where(bad, err / np.maximum(allow, 1e-300), -1))), err.shape)
        raise AssertionError(
            f"{what}: {int(bad.sum())} {kind} entries outside the gate (worst ratio {worst:.3e}; "
            f"e.g. at {tuple(int(v) for v in i)}: value {float(g[i]):.17g} oracle {float(ref[i]):.17g} "
            f"bound {float(bound[i]):.3e})")


def check_source(g, ref, bound, what):
    _check(g, ref, bound, SRC_TOL, 0.0, what, "source")


def check_jac(g, ref, bound, what):
    _check(g, ref, bound, JAC_TOL, JAC_ABS, what, "Jacobian")


# ---------------------------------------------------------------------------
# reports: literal errors and the paper's norms


def literal_report(g, ref, bound, tol, floor=0.0):
    """The literal relative test |g - ref| <= tol |ref| + floor, entry by
    entry: the largest relative error, the number of entries that fail it
    and the running-error condition number kappa = b / (u |ref|) of each."""
    g = np.asarray(g, dtype=np.float64)
    a = np.abs(ref)
    err = np.abs(g - ref)
    fail = err > tol * a + floor
    nzr = a > 0
    rel = np.where(nzr, err / np.where(nzr, a, 1.0), np.where(err > 0, np.inf, 0.0))
    kap = bound[fail] / (U_ROUND * np.maximum(a[fail], 1e-300))
    return {"max_rel_err": float(np.max(rel)) if rel.size else 0.0,
            "n_entries": int(ref.size), "n_literal_fail": int(fail.sum()),
            "literal_fail_kappa": sorted(float(k) for k in kap)[-10:],
            "n_widened": int(np.sum(bound > (tol / 100.0) * a))}


def e_x(g, ref):
    """Sec. 3.2 relative error norm: max |ref - g| / (1e-10 + 1e-6 |ref|)."""
    err = np.abs(np.asarray(ref) - np.asarray(g))
    return float(np.max(err / (1e-10 + 1e-6 * np.abs(ref)))) if err.size else 0.0


def e_c(Jg, Jref, C):
    """Sec. 3.3 filtered relative error: per state the Frobenius norm of the
    relative error over entries with |J_ref| >= T / C, T the Frobenius norm
    of the reference over all states; then the Frobenius norm over states.
    Jg, Jref: [n, N, N]."""
    T = np.sqrt(np.sum(Jref.astype(np.float64) ** 2))
    keep = np.abs(Jref) >= T / C
    rel = np.where(keep, (Jg - Jref) / np.where(keep, Jref, 1.0), 0.0)
    per_state = np.sqrt(np.sum(rel ** 2, axis=(1, 2)))
    return float(np.sqrt(np.sum(per_state ** 2)))


def e_l(Jg, Jref):
    """Sec. 3.3 LAPACK-style error: per state ||Jg - Jref||_F / ||Jref||_F,
    then the Frobenius norm over states."""
    num = np.sqrt(np.sum((Jg - Jref) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(Jref ** 2, axis=(1, 2)))
    return float(np.sqrt(np.sum((num / den) ** 2)))


def accuracy_report(f_g, f_ref, f_bound, J_g, J_ref, J_bound):
    """Source terms and Jacobian of the same states ([n, N] and [n, N, N]):
    the literal reports, E_X of dT/dt, dS/dt and dn/dt, E_C at C = 1e15 and
    1e20, E_L."""
    return {"source": literal_report(f_g, f_ref, f_bound, SRC_TOL),
            "jacobian": literal_report(J_g, J_ref, J_bound, JAC_TOL, JAC_ABS),
            "E_X_dTdt": e_x(f_g[:, 0], f_ref[:, 0]), "E_X_dSdt": e_x(f_g[:, 1], f_ref[:, 1]),
            "E_X_dndt": e_x(f_g[:, 2:], f_ref[:, 2:]),
            "E_C_1e20": e_c(J_g, J_ref, 1e20), "E_C_1e15": e_c(J_g, J_ref, 1e15),
            "E_L": e_l(J_g, J_ref)}
