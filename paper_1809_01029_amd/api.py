"""Python binding of the C-ABI in ``include/pjac.h`` (argument marshalling only).

Every evaluation runs in the HIP kernels of ``libpjac.so``; this module only
checks tensor shapes, dtypes and devices, allocates outputs with torch when
the caller does not pass them, and hands raw device pointers and the current
HIP stream to the library.  If the library has not been built the import of
this module fails: there is no fallback.

Layouts (paper Sec. 2.1): ``"F"`` keeps each variable of all states
contiguous, ``"C"`` keeps each state contiguous.

=========================  =====================  ======================
array                      layout "F" shape       layout "C" shape
=========================  =====================  ======================
state, dstate              (N, n)                 (n, N)
param                      (n,)                   (n,)
sparse Jacobian values     (nnz, n)               (n, nnz)
dense Jacobian             (N, N, n) as [j, i, s] (n, N, N) as [s, i, j]
=========================  =====================  ======================
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpjac.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_01029_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_lib.pj_mech_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_P)]
_lib.pj_mech_load.restype = ctypes.c_int
_lib.pj_mech_parse.argtypes = [ctypes.c_char_p, ctypes.POINTER(_P)]
_lib.pj_mech_parse.restype = ctypes.c_int
_lib.pj_mech_load_ex.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(_P)]
_lib.pj_mech_load_ex.restype = ctypes.c_int
_lib.pj_mech_parse_ex.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(_P)]
_lib.pj_mech_parse_ex.restype = ctypes.c_int
_lib.pj_mech_options.argtypes = [_P]
_lib.pj_mech_options.restype = ctypes.c_int
_lib.pj_mech_jac_pattern_ccs.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                         ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
_lib.pj_mech_jac_pattern_ccs.restype = ctypes.c_int
_lib.pj_mech_upload.argtypes = [_P]
_lib.pj_mech_upload.restype = ctypes.c_int
_lib.pj_mech_free.argtypes = [_P]
_lib.pj_mech_free.restype = None
for _f in ("pj_mech_n_species", "pj_mech_n_reactions", "pj_mech_state_size"):
    getattr(_lib, _f).argtypes = [_P]
    getattr(_lib, _f).restype = ctypes.c_int
_lib.pj_mech_jac_pattern.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                     ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
_lib.pj_mech_jac_pattern.restype = ctypes.c_int
_lib.pj_eval_source.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P]
_lib.pj_eval_source.restype = ctypes.c_int
_lib.pj_eval_jacobian_sparse.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P, _P]
_lib.pj_eval_jacobian_sparse.restype = ctypes.c_int
_lib.pj_eval_jacobian_dense.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P, _P]
_lib.pj_eval_jacobian_dense.restype = ctypes.c_int
_lib.pj_eval_adjoint.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P, _P, _P, _P]
_lib.pj_eval_adjoint.restype = ctypes.c_int
_lib.pj_calibrate_fp64.argtypes = [ctypes.c_int, _I64, ctypes.c_int, _P, _P, _P]
_lib.pj_calibrate_fp64.restype = ctypes.c_int
_lib.pj_eval_source_arrhenius.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P, _P]
_lib.pj_eval_source_arrhenius.restype = ctypes.c_int
_lib.pj_eval_adjoint_arrhenius.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P, _P, _P, _P, _P]
_lib.pj_eval_adjoint_arrhenius.restype = ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)
_lib.pj_mech_set_arrhenius.argtypes = [_P, _DP, _DP, _DP]
_lib.pj_mech_set_arrhenius.restype = ctypes.c_int
_lib.pj_mech_get_arrhenius.argtypes = [_P, _DP, _DP, _DP]
_lib.pj_mech_get_arrhenius.restype = ctypes.c_int
_lib.pj_batch_create.argtypes = [ctypes.POINTER(_P)]
_lib.pj_batch_create.restype = ctypes.c_int
_lib.pj_batch_free.argtypes = [_P]
_lib.pj_batch_free.restype = None
_lib.pj_batch_add.argtypes = [_P, _P, _I64, _P, _P, _P, _P, _P, _P]
_lib.pj_batch_add.restype = ctypes.c_int
_lib.pj_batch_clear.argtypes = [_P]
_lib.pj_batch_clear.restype = ctypes.c_int
_lib.pj_batch_size.argtypes = [_P]
_lib.pj_batch_size.restype = ctypes.c_int
_lib.pj_batch_set_launch.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
_lib.pj_batch_set_launch.restype = ctypes.c_int
_lib.pj_batch_launch_shape.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.pj_batch_launch_shape.restype = ctypes.c_int
_lib.pj_batch_segment_states.argtypes = [_P, ctypes.c_int, ctypes.c_int]
_lib.pj_batch_segment_states.restype = ctypes.c_int
_lib.pj_batch_eval.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P]
_lib.pj_batch_eval.restype = ctypes.c_int
_lib.pj_batch_eval_noalloc.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P]
_lib.pj_batch_eval_noalloc.restype = ctypes.c_int
_lib.pj_batch_eval_graph.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P]
_lib.pj_batch_eval_graph.restype = ctypes.c_int
_lib.pj_batch_autotune.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_float)]
_lib.pj_batch_autotune.restype = ctypes.c_int
_lib.pj_batch_set_strategy.argtypes = [_P, ctypes.c_int, ctypes.c_int]
_lib.pj_batch_set_strategy.restype = ctypes.c_int
_lib.pj_batch_strategy.argtypes = [_P, ctypes.c_int]
_lib.pj_batch_strategy.restype = ctypes.c_int
_lib.pj_batch_last_error.argtypes = []
_lib.pj_batch_last_error.restype = ctypes.c_char_p
_lib.pj_mech_set_waves_per_state.argtypes = [_P, ctypes.c_int]
_lib.pj_mech_set_waves_per_state.restype = ctypes.c_int
_lib.pj_mech_waves_per_state.argtypes = [_P, ctypes.c_int]
_lib.pj_mech_waves_per_state.restype = ctypes.c_int
_lib.pj_mech_set_launch.argtypes = [_P, ctypes.c_int, ctypes.c_int]
_lib.pj_mech_set_launch.restype = ctypes.c_int
_lib.pj_mech_launch_shape.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.pj_mech_launch_shape.restype = ctypes.c_int
_lib.pj_mech_set_dense_unroll.argtypes = [_P, ctypes.c_int]
_lib.pj_mech_set_dense_unroll.restype = ctypes.c_int
_lib.pj_mech_dense_unroll.argtypes = [_P]
_lib.pj_mech_dense_unroll.restype = ctypes.c_int
_lib.pj_mech_autotune.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P,
                                  ctypes.c_int, _P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_float)]
_lib.pj_mech_autotune.restype = ctypes.c_int
_lib.pj_mech_autotune_adjoint.argtypes = [_P, ctypes.c_int, ctypes.c_int, _I64, _P, _P, _P, _P, _P, ctypes.c_int,
                                          _P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_float)]
_lib.pj_mech_autotune_adjoint.restype = ctypes.c_int
_lib.pj_mech_lds_bytes.argtypes = [_P, ctypes.c_int]
_lib.pj_mech_lds_bytes.restype = _I64
_lib.pj_last_error.argtypes = []
_lib.pj_last_error.restype = ctypes.c_char_p

CONP, CONV = 0, 1
LAYOUT_F, LAYOUT_C = 0, 1
FORMS = {"conp": CONP, "conv": CONV}
LAYOUTS = {"F": LAYOUT_F, "C": LAYOUT_C}
STATUS = {0: "PJ_OK", 1: "PJ_E_INVALID", 2: "PJ_E_PARSE", 3: "PJ_E_UNBALANCED", 4: "PJ_E_DEVICE",
          5: "PJ_E_NOMEM", 6: "PJ_E_UNSUPPORTED"}


class PjError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.pj_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def _check(st: int, where: str):
    if st != 0:
        raise PjError(st, where)


def library() -> ctypes.CDLL:
    return _lib


OPT_APPROX_JACOBIAN, OPT_CCS, OPT_LINEAR_SEARCH, OPT_DETERMINISTIC = 1, 2, 4, 8


class Mechanism:
    """A mechanism description loaded by the library (pj_mech_load_ex), or
    only parsed on the host (``upload=False``, pj_mech_parse_ex).  ``options``:
    OPT_APPROX_JACOBIAN, OPT_CCS, OPT_LINEAR_SEARCH, OPT_DETERMINISTIC (bitwise or)."""

    def __init__(self, path: str, upload: bool = True, options: int = 0):
        h = _P()
        fn = _lib.pj_mech_load_ex if upload else _lib.pj_mech_parse_ex
        _check(fn(os.fsencode(path), int(options), ctypes.byref(h)), "pj_mech_load_ex" if upload else "pj_mech_parse_ex")
        self.options = int(options)
        self._h = h
        self.path = path
        self.n_species = _lib.pj_mech_n_species(h)
        self.n_reactions = _lib.pj_mech_n_reactions(h)
        self.N = _lib.pj_mech_state_size(h)
        nnz = _I64()
        rp = ctypes.POINTER(ctypes.c_int32)()
        ci = ctypes.POINTER(ctypes.c_int32)()
        _check(_lib.pj_mech_jac_pattern(h, ctypes.byref(nnz), ctypes.byref(rp), ctypes.byref(ci)),
               "pj_mech_jac_pattern")
        self.nnz = int(nnz.value)
        self.row_ptr = np.ctypeslib.as_array(rp, shape=(self.N + 1,)).astype(np.int64)
        self.col_idx = np.ctypeslib.as_array(ci, shape=(self.nnz,)).astype(np.int64)
        cp = ctypes.POINTER(ctypes.c_int32)()
        ri = ctypes.POINTER(ctypes.c_int32)()
        _check(_lib.pj_mech_jac_pattern_ccs(h, ctypes.byref(nnz), ctypes.byref(cp), ctypes.byref(ri)),
               "pj_mech_jac_pattern_ccs")
        self.col_ptr = np.ctypeslib.as_array(cp, shape=(self.N + 1,)).astype(np.int64)
        self.row_idx = np.ctypeslib.as_array(ri, shape=(self.nnz,)).astype(np.int64)

    def upload(self):
        _check(_lib.pj_mech_upload(self._h), "pj_mech_upload")

    @property
    def handle(self):
        return self._h

    def pattern_dense(self) -> np.ndarray:
        P = np.zeros((self.N, self.N), dtype=bool)
        rows = np.repeat(np.arange(self.N), np.diff(self.row_ptr))
        P[rows, self.col_idx] = True
        return P

    def set_waves_per_state(self, w: int):
        _check(_lib.pj_mech_set_waves_per_state(self._h, int(w)), "pj_mech_set_waves_per_state")

    def set_launch(self, states_per_group: int = 0, waves_per_group: int = 0):
        _check(_lib.pj_mech_set_launch(self._h, int(states_per_group), int(waves_per_group)),
               "pj_mech_set_launch")

    def set_dense_unroll(self, entries: int = 0):
        """Map reads in flight per lane in the dense output (8 or 16; 0: the
        default, 16), pj_mech_set_dense_unroll."""
        _check(_lib.pj_mech_set_dense_unroll(self._h, int(entries)), "pj_mech_set_dense_unroll")

    def dense_unroll(self) -> int:
        return _lib.pj_mech_dense_unroll(self._h)

    def launch_shape(self, mode: int = 1):
        """(states per workgroup, waves per workgroup) of mode 0 (source),
        1 (sparse Jacobian) or 2 (dense Jacobian)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        if _lib.pj_mech_launch_shape(self._h, int(mode), ctypes.byref(a), ctypes.byref(b)) != 0:
            raise PjError(1, "pj_mech_launch_shape")
        return a.value, b.value

    def arrhenius(self):
        """(ln A, b, Ea/R) of every reaction, description order (k_inf for falloff)."""
        nr = self.n_reactions
        a, b, t = np.zeros(nr), np.zeros(nr), np.zeros(nr)
        dp = lambda x: x.ctypes.data_as(_DP)
        _check(_lib.pj_mech_get_arrhenius(self._h, dp(a), dp(b), dp(t)), "pj_mech_get_arrhenius")
        return a, b, t

    def set_arrhenius(self, lnA=None, b=None, theta=None):
        """pj_mech_set_arrhenius: replace any of the three parameter arrays
        (length n_reactions, description order); synchronous."""
        nr = self.n_reactions
        keep = []

        def arr(x):
            if x is None:
                return None
            x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
            if x.shape[0] != nr:
                raise ValueError(f"expected {nr} values")
            keep.append(x)
            return x.ctypes.data_as(_DP)
        _check(_lib.pj_mech_set_arrhenius(self._h, arr(lnA), arr(b), arr(theta)), "pj_mech_set_arrhenius")

    def waves_per_state(self, jacobian: bool = False) -> int:
        return _lib.pj_mech_waves_per_state(self._h, 1 if jacobian else 0)

    def lds_bytes(self, jacobian: bool = False) -> int:
        return int(_lib.pj_mech_lds_bytes(self._h, 1 if jacobian else 0))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pj_mech_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def load_mechanism(path: str, options: int = 0) -> Mechanism:
    return Mechanism(path, upload=True, options=options)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t: torch.Tensor, shape: Tuple[int, ...], name: str, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name} must be on the mechanism's CUDA/HIP device")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _n_states(mech: Mechanism, state: torch.Tensor, layout: str) -> int:
    if state.dim() != 2:
        raise ValueError("state must be 2-D")
    return int(state.shape[1] if layout == "F" else state.shape[0])


def _state_shape(mech, n, layout):
    return (mech.N, n) if layout == "F" else (n, mech.N)


def eval_source(mech: Mechanism, state: torch.Tensor, param: torch.Tensor, form: str = "conp",
                layout: str = "F", out: Optional[torch.Tensor] = None, stream=None,
                arrhenius: Optional[torch.Tensor] = None) -> torch.Tensor:
    """pj_eval_source: dPhi/dt for every state.  ``arrhenius``: this call's
    (ln A, b, Ea/R) as a (3, n_reactions) float64 device tensor in
    description order (pj_eval_source_arrhenius), else the mechanism's."""
    n = _n_states(mech, state, layout)
    _need(state, _state_shape(mech, n, layout), "state", None)
    _need(param, (n,), "param", state.device)
    if out is None:
        out = torch.empty_like(state)
    _need(out, _state_shape(mech, n, layout), "out", state.device)
    if arrhenius is not None:
        _need(arrhenius, (3, mech.n_reactions), "arrhenius", state.device)
        _check(_lib.pj_eval_source_arrhenius(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state),
                                             _ptr(param), _ptr(arrhenius), _ptr(out), _stream(stream)),
               "pj_eval_source_arrhenius")
        return out
    _check(_lib.pj_eval_source(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state), _ptr(param),
                               _ptr(out), _stream(stream)), "pj_eval_source")
    return out


def eval_jacobian_sparse(mech: Mechanism, state: torch.Tensor, param: torch.Tensor, form: str = "conp",
                         layout: str = "F", out: Optional[torch.Tensor] = None,
                         dstate: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """pj_eval_jacobian_sparse: CSR values on the mechanism's pattern
    (``mech.row_ptr``, ``mech.col_idx``); optionally fused source terms into
    ``dstate``."""
    n = _n_states(mech, state, layout)
    _need(state, _state_shape(mech, n, layout), "state", None)
    _need(param, (n,), "param", state.device)
    shape = (mech.nnz, n) if layout == "F" else (n, mech.nnz)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=state.device)
    _need(out, shape, "out", state.device)
    if dstate is not None:
        _need(dstate, _state_shape(mech, n, layout), "dstate", state.device)
    _check(_lib.pj_eval_jacobian_sparse(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state),
                                        _ptr(param), _ptr(out), _ptr(dstate), _stream(stream)),
           "pj_eval_jacobian_sparse")
    return out


def eval_jacobian_dense(mech: Mechanism, state: torch.Tensor, param: torch.Tensor, form: str = "conp",
                        layout: str = "F", out: Optional[torch.Tensor] = None,
                        dstate: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """pj_eval_jacobian_dense: the full N x N Jacobian of every state
    (layout "C": [s, i, j]; layout "F": [j, i, s])."""
    n = _n_states(mech, state, layout)
    _need(state, _state_shape(mech, n, layout), "state", None)
    _need(param, (n,), "param", state.device)
    N = mech.N
    shape = (N, N, n) if layout == "F" else (n, N, N)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=state.device)
    _need(out, shape, "out", state.device)
    if dstate is not None:
        _need(dstate, _state_shape(mech, n, layout), "dstate", state.device)
    _check(_lib.pj_eval_jacobian_dense(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state),
                                       _ptr(param), _ptr(out), _ptr(dstate), _stream(stream)),
           "pj_eval_jacobian_dense")
    return out


MODES = {"source": 0, "sparse": 1, "dense": 2, "adjoint": 3}


def eval_adjoint(mech: Mechanism, state: torch.Tensor, param: torch.Tensor, v: torch.Tensor,
                 form: str = "conp", layout: str = "F", jtv: Optional[torch.Tensor] = None,
                 grad: Optional[torch.Tensor] = None, with_grad: bool = True,
                 dstate: Optional[torch.Tensor] = None, stream=None,
                 arrhenius: Optional[torch.Tensor] = None):
    """pj_eval_adjoint: (J^T v per state in the state layout, batch-summed
    d(v . dPhi/dt)/d(ln A, b, Ea/R) as a (3, n_reactions) tensor in
    description order, or None when ``with_grad`` is False).  ``arrhenius``:
    this call's parameters as in eval_source (pj_eval_adjoint_arrhenius)."""
    n = _n_states(mech, state, layout)
    _need(state, _state_shape(mech, n, layout), "state", None)
    _need(param, (n,), "param", state.device)
    _need(v, _state_shape(mech, n, layout), "v", state.device)
    if jtv is None:
        jtv = torch.empty_like(state)
    _need(jtv, _state_shape(mech, n, layout), "jtv", state.device)
    if with_grad:
        if grad is None:
            grad = torch.empty((3, mech.n_reactions), dtype=torch.float64, device=state.device)
        _need(grad, (3, mech.n_reactions), "grad", state.device)
    else:
        grad = None
    if dstate is not None:
        _need(dstate, _state_shape(mech, n, layout), "dstate", state.device)
    if arrhenius is not None:
        _need(arrhenius, (3, mech.n_reactions), "arrhenius", state.device)
        _check(_lib.pj_eval_adjoint_arrhenius(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state),
                                              _ptr(param), _ptr(arrhenius), _ptr(v), _ptr(jtv), _ptr(grad),
                                              _ptr(dstate), _stream(stream)), "pj_eval_adjoint_arrhenius")
        return jtv, grad
    _check(_lib.pj_eval_adjoint(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state), _ptr(param),
                                _ptr(v), _ptr(jtv), _ptr(grad), _ptr(dstate), _stream(stream)),
           "pj_eval_adjoint")
    return jtv, grad


def calibrate_fp64(fn: str, x: torch.Tensor, reps: int = 16, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """pj_calibrate_fp64: sum over r < reps of f(x + r 1e-3) per element, f
    one of "exp", "log", "log10" or "none" (the loop alone)."""
    code = {"exp": 0, "log": 1, "log10": 2, "none": 3}[fn]
    if out is None:
        out = torch.empty_like(x)
    _need(x, (x.numel(),), "x", None)
    _need(out, (x.numel(),), "out", x.device)
    _check(_lib.pj_calibrate_fp64(code, x.numel(), int(reps), _ptr(x), _ptr(out), _stream(stream)),
           "pj_calibrate_fp64")
    return out


class SourceTerms(torch.autograd.Function):
    """dPhi/dt as a differentiable function of the states and of the
    Arrhenius parameters (ln A, b, Ea/R): forward runs
    pj_eval_source_arrhenius with the given parameters, backward runs
    pj_eval_adjoint_arrhenius with the same (saved) parameters, so each graph
    differentiates at its own parameters; the mechanism's tables are never
    written and the host never waits.  The parameter P (CONP) or V (CONV)
    gets no gradient."""

    @staticmethod
    def forward(ctx, state, param, lnA, b, theta, mech, form, layout):
        arr = torch.stack([lnA.detach(), b.detach(), theta.detach()]).to(
            device=state.device, dtype=torch.float64).contiguous()
        ctx.mech, ctx.form, ctx.layout = mech, form, layout
        ctx.save_for_backward(state, param, arr)
        return eval_source(mech, state, param, form, layout, arrhenius=arr)

    @staticmethod
    def backward(ctx, v):
        state, param, arr = ctx.saved_tensors
        jtv, grad = eval_adjoint(ctx.mech, state, param, v.contiguous(), ctx.form, ctx.layout, arrhenius=arr)
        return jtv, None, grad[0], grad[1], grad[2], None, None, None


def source_terms(mech: Mechanism, state: torch.Tensor, param: torch.Tensor, lnA: torch.Tensor,
                 b: torch.Tensor, theta: torch.Tensor, form: str = "conp", layout: str = "F") -> torch.Tensor:
    """Differentiable source terms (see SourceTerms)."""
    return SourceTerms.apply(state, param, lnA, b, theta, mech, form, layout)


def autotune(mech: Mechanism, state: torch.Tensor, param: torch.Tensor, form: str = "conp",
             layout: str = "F", mode: str = "sparse", reps: int = 2, stream=None):
    """pj_mech_autotune: time every launch shape of ``mode`` ("source",
    "sparse", "dense", "adjoint") on this batch and keep the fastest for that mode.
    Returns (states per workgroup, waves per workgroup, ms per launch).
    Scratch outputs are allocated here and discarded."""
    n = _n_states(mech, state, layout)
    _need(state, _state_shape(mech, n, layout), "state", None)
    _need(param, (n,), "param", state.device)
    m = MODES[mode]
    S, W, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    if m == 3:
        # the adjoint: time with v = the states themselves and the parameter sums
        jtv = torch.empty_like(state)
        grad = torch.empty((3, mech.n_reactions), dtype=torch.float64, device=state.device)
        _check(_lib.pj_mech_autotune_adjoint(mech.handle, FORMS[form], LAYOUTS[layout], n, _ptr(state),
                                             _ptr(param), _ptr(state), _ptr(jtv), _ptr(grad), int(reps),
                                             _stream(stream), ctypes.byref(S), ctypes.byref(W), ctypes.byref(ms)),
               "pj_mech_autotune_adjoint")
        return S.value, W.value, ms.value
    dstate = torch.empty_like(state)
    if m == 0:
        out = dstate
    elif m == 1:
        out = torch.empty((mech.nnz, n) if layout == "F" else (n, mech.nnz), dtype=torch.float64,
                          device=state.device)
    else:
        out = torch.empty((mech.N, mech.N, n) if layout == "F" else (n, mech.N, mech.N), dtype=torch.float64,
                          device=state.device)
    _check(_lib.pj_mech_autotune(mech.handle, m, FORMS[form], LAYOUTS[layout], n, _ptr(state), _ptr(param),
                                 _ptr(out), _ptr(dstate) if m else None, int(reps), _stream(stream),
                                 ctypes.byref(S), ctypes.byref(W), ctypes.byref(ms)), "pj_mech_autotune")
    return S.value, W.value, ms.value


class Batch:
    """A ragged multi-mechanism batch (pj_batch_*): segments of states of
    different mechanisms evaluated by one launch, or by a captured HIP graph.
    The tensors of every segment are kept referenced here while the batch
    lives.  ``mode``: "source", "sparse" or "adjoint"."""

    def __init__(self):
        h = _P()
        _check(_lib.pj_batch_create(ctypes.byref(h)), "pj_batch_create")
        self._h = h
        self._keep = []

    def _bcheck(self, st, where):
        if st != 0:
            raise PjError(st, f"{where}: {_lib.pj_batch_last_error().decode()}")

    def add(self, mech: Mechanism, state: torch.Tensor, param: torch.Tensor, layout: str,
            out: Optional[torch.Tensor] = None, dstate: Optional[torch.Tensor] = None,
            v: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
        n = _n_states(mech, state, layout)
        _need(state, _state_shape(mech, n, layout), "state", None)
        _need(param, (n,), "param", state.device)
        self._keep.append((mech, state, param, out, dstate, v, grad))
        self._bcheck(_lib.pj_batch_add(self._h, mech.handle, n, _ptr(state), _ptr(param), _ptr(out), _ptr(dstate),
                                       _ptr(v), _ptr(grad)), "pj_batch_add")

    def clear(self):
        self._keep = []
        self._bcheck(_lib.pj_batch_clear(self._h), "pj_batch_clear")

    def __len__(self):
        return _lib.pj_batch_size(self._h)

    def set_launch(self, mode: str, states_per_group: int = 0, waves_per_group: int = 0):
        self._bcheck(_lib.pj_batch_set_launch(self._h, MODES[mode], states_per_group, waves_per_group),
                     "pj_batch_set_launch")

    def launch_shape(self, mode: str):
        a, b = ctypes.c_int(), ctypes.c_int()
        if _lib.pj_batch_launch_shape(self._h, MODES[mode], ctypes.byref(a), ctypes.byref(b)) != 0:
            raise PjError(1, "pj_batch_launch_shape")
        return a.value, b.value

    def segment_states(self, mode: str):
        """States per workgroup each segment takes in the persistent launch
        (pj_batch_segment_states)."""
        out = []
        for i in range(_lib.pj_batch_size(self._h)):
            v = _lib.pj_batch_segment_states(self._h, MODES[mode], i)
            if v < 0:
                raise PjError(1, "pj_batch_segment_states")
            out.append(v)
        return out

    def set_strategy(self, mode: str, per_segment: bool):
        """One persistent launch (False) or one launch per segment at each
        mechanism's own launch shape (True) for ``mode``."""
        self._bcheck(_lib.pj_batch_set_strategy(self._h, MODES[mode], int(bool(per_segment))),
                     "pj_batch_set_strategy")

    def strategy(self, mode: str) -> bool:
        return _lib.pj_batch_strategy(self._h, MODES[mode]) == 1

    def eval(self, mode: str, form: str = "conp", layout: str = "F", graph: bool = False, stream=None):
        f = _lib.pj_batch_eval_graph if graph else _lib.pj_batch_eval
        self._bcheck(f(self._h, MODES[mode], FORMS[form], LAYOUTS[layout], _stream(stream)),
                     "pj_batch_eval_graph" if graph else "pj_batch_eval")

    def eval_noalloc(self, mode: str, form: str = "conp", layout: str = "F", stream=None):
        """pj_batch_eval_noalloc: the persistent launch with the segment table
        in the library's fixed device array (no device allocation)."""
        self._bcheck(_lib.pj_batch_eval_noalloc(self._h, MODES[mode], FORMS[form], LAYOUTS[layout],
                                                _stream(stream)), "pj_batch_eval_noalloc")

    def autotune(self, mode: str, form: str = "conp", layout: str = "F", reps: int = 2, stream=None):
        """Keep the fastest of every persistent launch shape and one launch per
        segment; returns (S, W, ms), (0, 0, ms) for the per-segment launches."""
        S, W, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
        self._bcheck(_lib.pj_batch_autotune(self._h, MODES[mode], FORMS[form], LAYOUTS[layout], reps,
                                            _stream(stream), ctypes.byref(S), ctypes.byref(W), ctypes.byref(ms)),
                     "pj_batch_autotune")
        return S.value, W.value, ms.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pj_batch_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def dense_as_sij(jac: torch.Tensor, layout: str) -> torch.Tensor:
    """View a dense Jacobian output as [state, row, col]."""
    return jac if layout == "C" else jac.permute(2, 1, 0)


def sparse_to_dense(mech: Mechanism, vals: np.ndarray, layout: str) -> np.ndarray:
    """Host helper: sparse values (numpy, library layout; column order when
    the mechanism was loaded with OPT_CCS) -> dense [s, i, j]."""
    v = vals.T if layout == "F" else vals
    n = v.shape[0]
    out = np.zeros((n, mech.N, mech.N))
    if mech.options & OPT_CCS:
        cols = np.repeat(np.arange(mech.N), np.diff(mech.col_ptr))
        out[:, mech.row_idx, cols] = v
    else:
        rows = np.repeat(np.arange(mech.N), np.diff(mech.row_ptr))
        out[:, rows, mech.col_idx] = v
    return out
