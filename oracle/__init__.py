"""CPU oracle for the source terms and Jacobian (test infrastructure only).

A plain serial FP64 C++ evaluation (``oracle.cpp``) of the thermochemical
source terms and the analytical Jacobian of pyJac v2 (Curtis, Niemeyer & Sung,
arXiv:1809.01029, Sec. 2.2 and Sec. 3.4), loaded through ctypes.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it; the
GPU library never does.  It shares no code with the GPU library.

Arrays are row-major numpy float64: states ``x[n, N]`` with
``N = Ns + 1`` and ``x[s] = (T, V or P, n_1..n_{Ns-1})``, parameters ``p[n]``
(P for constant pressure, V for constant volume), Jacobians ``J[n, N, N]``
with ``J[s, i, j] = d(dPhi_i/dt)/dPhi_j``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CONP, CONV = 0, 1
_FORMS = {"conp": CONP, "conv": CONV, CONP: CONP, CONV: CONV}


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c++17",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        lib.ora_load.restype = P
        lib.ora_load.argtypes = [ctypes.c_char_p]
        lib.ora_free.argtypes = [P]
        lib.ora_ns.argtypes = [P]
        lib.ora_nr.argtypes = [P]
        lib.ora_thermo.argtypes = [P, ctypes.c_int, ctypes.c_double, D]
        lib.ora_components.argtypes = [P, ctypes.c_int, D, ctypes.c_double, D]
        lib.ora_source.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, D]
        lib.ora_jacobian.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, D]
        lib.ora_jacobian_cs.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, ctypes.c_double, D]
        lib.ora_jacobian_fd.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, ctypes.c_double, D]
        lib.ora_pattern.argtypes = [P, ctypes.POINTER(ctypes.c_ubyte)]
        lib.ora_jacobian_ex.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, D, ctypes.c_int]
        lib.ora_jacobian_cs_ex.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, ctypes.c_double, D, ctypes.c_int]
        lib.ora_pattern_ex.argtypes = [P, ctypes.POINTER(ctypes.c_ubyte), ctypes.c_int]
        lib.ora_adjoint.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, D, D, D, D]
        lib.ora_param_grad_cs.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, ctypes.c_double, D]
        lib.ora_jvp_cs.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, ctypes.c_double, D]
        lib.ora_source_ld.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D]
        lib.ora_jacobian_ld.argtypes = [P, ctypes.c_int, ctypes.c_long, D, D, D, ctypes.c_int]
        lib.ora_source_ops.argtypes = [P, ctypes.c_int, D, ctypes.c_double, D, D]
        _lib = lib
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One mechanism description loaded into the oracle."""

    def __init__(self, path: str):
        lib = _load()
        self._lib = lib
        self._h = lib.ora_load(path.encode())
        if not self._h:
            raise ValueError(f"oracle could not parse {path}")
        self.ns = lib.ora_ns(self._h)
        self.nr = lib.ora_nr(self._h)
        self.N = self.ns + 1

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_free(h)
            self._h = None

    def thermo(self, k: int, T: float):
        """(Cp/R, H/RT, S/R, dCp/R/dT, d(H/RT)/dT, d(S/R)/dT) of species k."""
        out = np.zeros(6)
        self._lib.ora_thermo(self._h, k, float(T), _d(out))
        return out

    def components(self, x, p: float, form="conp"):
        """Sub-components at one state (cf. the per-component unit tests of
        Sec. 2.3): dict of per-reaction kf, kr, c, Rf, Rr, q, and wdot, C,
        Tdot, Sdot, N (= sum e_k wdot_k), D (= sum [C]_k chat_k), Omega."""
        x = _f64(x)
        nr, ns = self.nr, self.ns
        out = np.zeros(6 * nr + 2 * ns + 5)
        self._lib.ora_components(self._h, _FORMS[form], _d(x), float(p), _d(out))
        r = out[: 6 * nr].reshape(nr, 6)
        t = out[6 * nr + 2 * ns:]
        return {"kf": r[:, 0], "kr": r[:, 1], "c": r[:, 2], "Rf": r[:, 3], "Rr": r[:, 4],
                "q": r[:, 5], "wdot": out[6 * nr: 6 * nr + ns],
                "C": out[6 * nr + ns: 6 * nr + 2 * ns], "Tdot": t[0], "Sdot": t[1],
                "N": t[2], "D": t[3], "Omega": t[4]}

    def source(self, x, p, form="conp", bound: bool = False):
        """Source terms [n, N]; with ``bound``, also the running error bound
        of every value (a first-order bound on |computed - exact|, in the
        value's units)."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        n = x.shape[0]
        f = np.zeros_like(x)
        b = np.zeros_like(x) if bound else None
        self._lib.ora_source(self._h, _FORMS[form], n, _d(x), _d(p), _d(f),
                             _d(b) if bound else None)
        return (f, b) if bound else f

    def jacobian(self, x, p, form="conp", bound: bool = False, approx: bool = False):
        """Analytical Jacobian [n, N, N] (with ``bound``, also the running
        error bound of every entry); ``approx``: the approximate form (the
        bath gas's moles held fixed against the other species')."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        n = x.shape[0]
        J = np.zeros((n, self.N, self.N))
        b = np.zeros_like(J) if bound else None
        self._lib.ora_jacobian_ex(self._h, _FORMS[form], n, _d(x), _d(p), _d(J),
                                  _d(b) if bound else None, int(approx))
        return (J, b) if bound else J

    def source_ld(self, x, p, form="conp"):
        """Source terms evaluated in long double, rounded to double."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        f = np.zeros_like(x)
        self._lib.ora_source_ld(self._h, _FORMS[form], x.shape[0], _d(x), _d(p), _d(f))
        return f

    def jacobian_ld(self, x, p, form="conp", approx: bool = False):
        """Analytical Jacobian evaluated in long double, rounded to double."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        J = np.zeros((x.shape[0], self.N, self.N))
        self._lib.ora_jacobian_ld(self._h, _FORMS[form], x.shape[0], _d(x), _d(p), _d(J), int(approx))
        return J

    def source_ops(self, x, p: float, form="conp", values: bool = False):
        """Arithmetic operations of one state's source terms as the oracle
        writes them, without the derivatives it forms along the way for the
        Jacobian and the parameter gradient, a transcendental of a repeated
        argument counted once: dict(flops = + - * / count, exp, log, log10)
        (and, with ``values``, the source terms of that evaluation)."""
        x = _f64(x).reshape(-1)
        out = np.zeros(4)
        f = np.zeros(self.N)
        self._lib.ora_source_ops(self._h, _FORMS[form], _d(x), float(p), _d(out), _d(f))
        ops = {"flops": int(out[0]), "exp": int(out[1]), "log": int(out[2]), "log10": int(out[3])}
        return (ops, f) if values else ops

    def jacobian_cs(self, x, p, form="conp", hrel: float = 1e-30, approx: bool = False):
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        J = np.zeros((x.shape[0], self.N, self.N))
        self._lib.ora_jacobian_cs_ex(self._h, _FORMS[form], x.shape[0], _d(x), _d(p), hrel, _d(J), int(approx))
        return J

    def jacobian_fd(self, x, p, form="conp", rel: float = 1e-6):
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        J = np.zeros((x.shape[0], self.N, self.N))
        self._lib.ora_jacobian_fd(self._h, _FORMS[form], x.shape[0], _d(x), _d(p), rel, _d(J))
        return J

    def adjoint(self, x, p, v, form="conp", bound: bool = False):
        """(J^T v per state [n, N], batch-summed d(v . dPhi/dt)/d(ln A, b, Ea/R)
        per reaction [3, nr] in description order), with the running error
        bounds of both if ``bound``."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        v = _f64(v).reshape(-1, self.N)
        n = x.shape[0]
        jtv = np.zeros_like(x)
        g = np.zeros((3, self.nr))
        js = np.zeros_like(x) if bound else None
        gs = np.zeros_like(g) if bound else None
        self._lib.ora_adjoint(self._h, _FORMS[form], n, _d(x), _d(p), _d(v), _d(jtv), _d(g),
                              _d(js) if bound else None, _d(gs) if bound else None)
        return (jtv, g, js, gs) if bound else (jtv, g)

    def param_grad_cs(self, x, p, v, form="conp", hrel: float = 1e-30):
        """Complex-step d(v . dPhi/dt)/d(ln A, b, Ea/R), summed over states."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        v = _f64(v).reshape(-1, self.N)
        g = np.zeros((3, self.nr))
        self._lib.ora_param_grad_cs(self._h, _FORMS[form], x.shape[0], _d(x), _d(p), _d(v), hrel, _d(g))
        return g

    def jvp_cs(self, x, p, u, form="conp", hstep: float = 1e-30):
        """Complex-step J u per state."""
        x = _f64(x).reshape(-1, self.N)
        p = _f64(p).reshape(-1)
        u = _f64(u).reshape(-1, self.N)
        out = np.zeros_like(x)
        self._lib.ora_jvp_cs(self._h, _FORMS[form], x.shape[0], _d(x), _d(p), _d(u), hstep, _d(out))
        return out

    def pattern(self, approx: bool = False) -> np.ndarray:
        P = np.zeros((self.N, self.N), dtype=np.uint8)
        self._lib.ora_pattern_ex(self._h, P.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), int(approx))
        return P.astype(bool)

    def csr(self, approx: bool = False):
        """The structural pattern as CSR (row_ptr[N+1], col_idx[nnz]), columns ascending."""
        P = self.pattern(approx)
        rows, cols = np.nonzero(P)
        row_ptr = np.zeros(self.N + 1, dtype=np.int64)
        np.add.at(row_ptr, rows + 1, 1)
        return np.cumsum(row_ptr), cols.astype(np.int64)
