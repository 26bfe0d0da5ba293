"""C-ABI contract on the host (no GPU): symbols, host-side mechanism
compilation (pattern) and error paths."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1809_01029_amd import synth
from conftest import TINY_SEEDS, tiny_file, workload_file

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pjac.h")


@pytest.fixture(scope="module")
def api():
    from paper_1809_01029_amd import api as a
    return a


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pj_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(api):
    lib = api.library()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("name", list(synth.WORKLOADS))
def test_pattern_matches_oracle_workloads(api, name, mech_dir):
    m, path = workload_file(name, mech_dir)
    mech = api.Mechanism(path, upload=False)
    assert mech.n_species == m.n_species and mech.n_reactions == m.n_reactions
    assert mech.N == m.n_species + 1
    np.testing.assert_array_equal(mech.pattern_dense(), oracle.Oracle(path).pattern())
    rp, ci = mech.row_ptr, mech.col_idx
    assert rp[0] == 0 and rp[-1] == mech.nnz and np.all(np.diff(rp) > 0)
    for i in range(mech.N):
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)


@pytest.mark.parametrize("seed", TINY_SEEDS)
@pytest.mark.parametrize("bath", [False, True])
def test_pattern_matches_oracle_tiny(api, seed, bath, mech_dir):
    kw = dict(bath_reactions=1, bath_efficiency=True) if bath else {}
    m, path = tiny_file(seed, mech_dir, **kw)
    mech = api.Mechanism(path, upload=False)
    np.testing.assert_array_equal(mech.pattern_dense(), oracle.Oracle(path).pattern())


def _write(tmp_path, text, name="m.pjm"):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def _status(api, path):
    h = ctypes.c_void_p()
    st = api.library().pj_mech_parse(os.fsencode(path), ctypes.byref(h))
    if st == 0:
        api.library().pj_mech_free(h)
    else:
        assert not h.value
    return st


def test_error_paths(api, tmp_path):
    lib = api.library()
    assert _status(api, str(tmp_path / "missing.pjm")) == 1          # PJ_E_INVALID
    assert _status(api, _write(tmp_path, "hello world")) == 2         # PJ_E_PARSE
    m = synth.make_mechanism(7, 10, 3, mix=synth.MixSpec(0.1, 0.2, 0.2), zipf=0.5)
    good = synth.dumps(m)
    assert _status(api, _write(tmp_path, good)) == 0
    assert _status(api, _write(tmp_path, good.replace("END", ""))) == 2
    # break the element balance of one reaction: change a product species
    bad = synth.loads(good)
    r = bad.reactions[0]
    sp, nu = r.prod[0]
    other = next(k for k in range(bad.n_species) if not np.array_equal(bad.comp[k], bad.comp[sp])
                 and k not in [s for s, _ in r.reac + r.prod])
    r.prod[0] = (other, nu)
    assert _status(api, _write(tmp_path, synth.dumps(bad))) == 3      # PJ_E_UNBALANCED
    # a species on both sides is outside what the kernels accept
    # (adding one species to both sides keeps the balance)
    both = synth.loads(good)
    r = next(r for r in both.reactions if len(r.reac) < 3 and len(r.prod) < 3)
    x = next(k for k in range(both.n_species) if k not in [s for s, _ in r.reac + r.prod])
    r.reac = r.reac + [(x, 1)]
    r.prod = r.prod + [(x, 1)]
    assert _status(api, _write(tmp_path, synth.dumps(both))) == 6      # PJ_E_UNSUPPORTED
    # NULL handling
    assert lib.pj_mech_n_species(None) == -1
    assert lib.pj_mech_state_size(None) == -1
    lib.pj_mech_free(None)
    h = ctypes.c_void_p()
    assert lib.pj_mech_load(None, ctypes.byref(h)) == 1
    assert lib.pj_mech_parse(os.fsencode(_write(tmp_path, good)), None) == 1


def test_eval_argument_checks_without_device(api, tmp_path):
    lib = api.library()
    m = synth.make_mechanism(7, 10, 3, mix=synth.MixSpec(0.1, 0.2, 0.2), zipf=0.5)
    mech = api.Mechanism(_write(tmp_path, synth.dumps(m)), upload=False)
    dummy = ctypes.c_void_p(16)
    # n_states == 0 is a no-op
    assert lib.pj_eval_source(mech.handle, 0, 0, 0, None, None, None, None) == 0
    # negative n, bad enums, NULL pointers, NULL handle, not uploaded
    assert lib.pj_eval_source(mech.handle, 0, 0, -1, dummy, dummy, dummy, None) == 1
    assert lib.pj_eval_source(mech.handle, 2, 0, 1, dummy, dummy, dummy, None) == 1
    assert lib.pj_eval_source(mech.handle, 0, 5, 1, dummy, dummy, dummy, None) == 1
    assert lib.pj_eval_source(mech.handle, 0, 0, 1, None, dummy, dummy, None) == 1
    assert lib.pj_eval_source(None, 0, 0, 1, dummy, dummy, dummy, None) == 1
    assert lib.pj_eval_jacobian_sparse(mech.handle, 0, 0, 1, dummy, dummy, None, None, None) == 1
    assert lib.pj_eval_jacobian_dense(mech.handle, 0, 0, 1, dummy, dummy, None, None, None) == 1
    assert lib.pj_eval_source(mech.handle, 0, 0, 1, dummy, dummy, dummy, None) == 1
    assert b"not uploaded" in lib.pj_last_error()
    assert lib.pj_mech_set_waves_per_state(mech.handle, 3) == 1
    assert lib.pj_mech_set_waves_per_state(mech.handle, 2) == 0
    assert lib.pj_mech_waves_per_state(mech.handle, 0) == 2
    assert lib.pj_mech_set_waves_per_state(mech.handle, 0) == 0


def test_launch_shape_and_autotune_argument_checks(api, tmp_path):
    lib = api.library()
    m = synth.make_mechanism(7, 10, 3, mix=synth.MixSpec(0.1, 0.2, 0.2), zipf=0.5)
    mech = api.Mechanism(_write(tmp_path, synth.dumps(m)), upload=False)
    h = mech.handle
    dummy = ctypes.c_void_p(16)
    # states per workgroup: powers of two up to 64; waves: 1 to 8
    for S in (1, 2, 4, 8, 16, 32, 64):
        assert lib.pj_mech_set_launch(h, S, 1) == 0
        assert mech.launch_shape(1) == (S, 1)
    for W in range(1, 9):
        assert lib.pj_mech_set_launch(h, 2, W) == 0
        assert mech.launch_shape(1) == (2, W)
    for S, W in ((3, 1), (128, 1), (-1, 1), (4, 9), (4, 16), (4, -1)):
        assert lib.pj_mech_set_launch(h, S, W) == 1
    assert lib.pj_mech_set_launch(h, 0, 0) == 0
    # autotune: argument errors are reported before any device work
    S, W, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    args = (0, 0, 16, dummy, dummy, dummy, None, 2, None, ctypes.byref(S), ctypes.byref(W), ctypes.byref(ms))
    assert lib.pj_mech_autotune(None, 1, *args) == 1
    assert lib.pj_mech_autotune(h, 3, *args) == 1
    assert b"bad mode" in lib.pj_last_error()
    bad_reps = (0, 0, 16, dummy, dummy, dummy, None, 0, None, None, None, None)
    assert lib.pj_mech_autotune(h, 1, *bad_reps) == 1
    no_states = (0, 0, 0, dummy, dummy, dummy, None, 2, None, None, None, None)
    assert lib.pj_mech_autotune(h, 1, *no_states) == 1
    assert lib.pj_mech_autotune(h, 1, *args) == 1
    assert b"not uploaded" in lib.pj_last_error()


def test_adjoint_and_arrhenius_argument_checks(api, tmp_path):
    lib = api.library()
    m = synth.make_mechanism(7, 10, 3, mix=synth.MixSpec(0.1, 0.2, 0.2), zipf=0.5)
    mech = api.Mechanism(_write(tmp_path, synth.dumps(m)), upload=False)
    h = mech.handle
    dummy = ctypes.c_void_p(16)
    # NULL v, NULL J^T v, not uploaded, bad enums
    assert lib.pj_eval_adjoint(h, 0, 0, 4, dummy, dummy, None, dummy, None, None, None) == 1
    assert b"NULL vector" in lib.pj_last_error()
    assert lib.pj_eval_adjoint(h, 0, 0, 4, dummy, dummy, dummy, None, None, None, None) == 1
    assert lib.pj_eval_adjoint(h, 2, 0, 4, dummy, dummy, dummy, dummy, None, None, None) == 1
    assert lib.pj_eval_adjoint(h, 0, 0, 4, dummy, dummy, dummy, dummy, None, None, None) == 1
    assert b"not uploaded" in lib.pj_last_error()
    assert lib.pj_eval_adjoint(None, 0, 0, 4, dummy, dummy, dummy, dummy, None, None, None) == 1
    # parameters round-trip on the host, in description order
    lnA, b, th = mech.arrhenius()
    np.testing.assert_array_equal(lnA, [r.lnA for r in m.reactions])
    np.testing.assert_array_equal(th, [r.theta for r in m.reactions])
    mech.set_arrhenius(lnA=lnA + 1.0)
    a2, b2, t2 = mech.arrhenius()
    np.testing.assert_array_equal(a2, lnA + 1.0)
    np.testing.assert_array_equal(b2, b)
    assert lib.pj_mech_set_arrhenius(None, None, None, None) == 1
    # the adjoint mode keeps at most 4 states per workgroup
    mech.set_launch(16, 1)
    assert mech.launch_shape(3)[0] <= 4
    # the dense output's map reads in flight: 8 or 16 (0: the default, 16)
    assert mech.dense_unroll() == 16
    mech.set_dense_unroll(8)
    assert mech.dense_unroll() == 8
    mech.set_dense_unroll(0)
    assert mech.dense_unroll() == 16
    for bad in (4, 12, 32, -1):
        assert lib.pj_mech_set_dense_unroll(mech.handle, bad) == 1
    assert lib.pj_mech_set_dense_unroll(None, 8) == 1 and lib.pj_mech_dense_unroll(None) == -1


def test_batch_argument_checks(api, tmp_path):
    lib = api.library()
    m = synth.make_mechanism(7, 10, 3, mix=synth.MixSpec(0.1, 0.2, 0.2), zipf=0.5)
    mech = api.Mechanism(_write(tmp_path, synth.dumps(m)), upload=False)
    dummy = ctypes.c_void_p(16)
    b = ctypes.c_void_p()
    assert lib.pj_batch_create(ctypes.byref(b)) == 0
    assert lib.pj_batch_size(b) == 0
    assert lib.pj_batch_launch_shape(b, 1, None, None) == -1     # empty
    assert lib.pj_batch_add(b, None, 4, dummy, dummy, dummy, None, None, None) == 1
    assert lib.pj_batch_add(b, mech.handle, -1, dummy, dummy, dummy, None, None, None) == 1
    assert lib.pj_batch_add(b, mech.handle, 4, dummy, dummy, dummy, None, None, None) == 0
    assert lib.pj_batch_size(b) == 1
    for mode, S, W in ((2, 1, 1), (1, 32, 1), (1, 3, 1), (1, 12, 1), (1, 1, 9), (1, 1, -1)):
        assert lib.pj_batch_set_launch(b, mode, S, W) == 1
    assert lib.pj_batch_set_launch(b, 1, 2, 4) == 0
    assert lib.pj_batch_set_launch(b, 1, 2, 7) == 0
    # per-segment states: -1 for a NULL batch, a bad mode or segment index
    assert lib.pj_batch_segment_states(None, 1, 0) == -1
    assert lib.pj_batch_segment_states(b, 2, 0) == -1
    assert lib.pj_batch_segment_states(b, 1, 1) == -1 and lib.pj_batch_segment_states(b, 1, -1) == -1
    # strategy: one persistent launch (0, the default) or one per segment (1)
    assert lib.pj_batch_strategy(b, 1) == 0
    assert lib.pj_batch_set_strategy(b, 1, 2) == 1
    assert lib.pj_batch_set_strategy(b, 2, 1) == 1
    assert lib.pj_batch_set_strategy(None, 1, 1) == 1
    assert lib.pj_batch_set_strategy(b, 1, 1) == 0 and lib.pj_batch_strategy(b, 1) == 1
    assert lib.pj_batch_set_strategy(b, 1, 0) == 0 and lib.pj_batch_strategy(b, 1) == 0
    assert lib.pj_batch_strategy(None, 1) == -1 and lib.pj_batch_strategy(b, 2) == -1
    # modes: 0, 1, 3 only; a mechanism that is not uploaded is reported by segment
    assert lib.pj_batch_eval(b, 2, 0, 0, None) == 1
    assert lib.pj_batch_eval(b, 1, 0, 0, None) == 1
    assert b"segment 0" in lib.pj_batch_last_error() and b"not uploaded" in lib.pj_batch_last_error()
    assert lib.pj_batch_clear(b) == 0 and lib.pj_batch_size(b) == 0
    lib.pj_batch_free(b)
    lib.pj_batch_free(None)


@pytest.mark.parametrize("name", ["ns13", "ns53", "ns111", "ns360"])
def test_approximate_pattern_matches_oracle(api, name, mech_dir):
    m, path = workload_file(name, mech_dir)
    mech = api.Mechanism(path, upload=False, options=api.OPT_APPROX_JACOBIAN)
    assert mech.options == api.OPT_APPROX_JACOBIAN
    np.testing.assert_array_equal(mech.pattern_dense(), oracle.Oracle(path).pattern(approx=True))


@pytest.mark.parametrize("seed", TINY_SEEDS)
def test_approximate_pattern_matches_oracle_tiny(api, seed, mech_dir):
    m, path = tiny_file(seed, mech_dir, bath_reactions=1, bath_efficiency=True)
    mech = api.Mechanism(path, upload=False, options=api.OPT_APPROX_JACOBIAN)
    np.testing.assert_array_equal(mech.pattern_dense(), oracle.Oracle(path).pattern(approx=True))


def test_column_order_arrays_and_options(api, mech_dir, tmp_path):
    m, path = workload_file("ns53", mech_dir)
    mech = api.Mechanism(path, upload=False, options=api.OPT_CCS)
    P = np.zeros((mech.N, mech.N), dtype=bool)
    cols = np.repeat(np.arange(mech.N), np.diff(mech.col_ptr))
    P[mech.row_idx, cols] = True
    np.testing.assert_array_equal(P, mech.pattern_dense())
    for c in range(mech.N):   # rows ascending within each column
        assert np.all(np.diff(mech.row_idx[mech.col_ptr[c]:mech.col_ptr[c + 1]]) > 0)
    # CCS of a dense matrix recovers it through sparse_to_dense
    rng = np.random.default_rng(0)
    D = rng.standard_normal((2, mech.N, mech.N)) * mech.pattern_dense()
    vals = D[:, mech.row_idx, cols]
    np.testing.assert_array_equal(api.sparse_to_dense(mech, vals, "C"), D)
    lib = api.library()
    h = ctypes.c_void_p()
    assert lib.pj_mech_parse_ex(os.fsencode(path), 16, ctypes.byref(h)) == 1
    assert b"option" in lib.pj_last_error()
    det = api.Mechanism(path, upload=False, options=api.OPT_DETERMINISTIC | api.OPT_CCS)
    assert lib.pj_mech_options(det._h) == api.OPT_DETERMINISTIC | api.OPT_CCS
    assert lib.pj_mech_options(None) == -1


@pytest.mark.parametrize("bath", [False, True])
def test_pattern_matches_oracle_all_types(api, bath, mech_dir):
    from conftest import TYPES_SEEDS, types_file
    for seed in TYPES_SEEDS:
        m, path = types_file(seed, mech_dir, bath=bath)
        mech = api.Mechanism(path, upload=False)
        np.testing.assert_array_equal(mech.pattern_dense(), oracle.Oracle(path).pattern())


def test_error_paths_of_further_reaction_types(api, tmp_path):
    from conftest import TYPES_SEEDS, types_file
    m, _ = types_file(TYPES_SEEDS[0], tmp_path)
    good = synth.dumps(m)
    assert _status(api, _write(tmp_path, good)) == 0

    def edited(fn):
        mm = synth.loads(good)
        fn(mm)
        return _status(api, _write(tmp_path, synth.dumps(mm)))

    def first(mm, t):
        return next(r for r in mm.reactions if r.type == t)

    def pl_descending(mm):
        r = first(mm, "PLOG")
        r.plog = r.plog[::-1]

    def pl_too_long(mm):
        r = first(mm, "PLOG")
        r.plog = [(synth.ATM * (1 + k), 30.0, 0.0, 0.0) for k in range(65)]

    def cheb_bad_range(mm):
        r = first(mm, "CHEB")
        (t0, t1, p0, p1), c = r.cheb
        r.cheb = ((t1, t0, p0, p1), c)

    def cheb_too_big(mm):
        r = first(mm, "CHEB")
        r.cheb = (r.cheb[0], [[1.0] * 2 for _ in range(17)])

    def chemact_on_elem(mm):
        first(mm, "ELEM").chemact = True

    def sri_bad(mm):
        r = first(mm, "SRI")
        r.sri = (0.5, 100.0, -3.0, 1.0, 0.0)

    def eff_on_plog(mm):
        first(mm, "PLOG").eff = [(0, 2.0)]

    assert edited(pl_descending) == 2          # PJ_E_PARSE
    assert edited(pl_too_long) == 6            # PJ_E_UNSUPPORTED
    assert edited(cheb_bad_range) == 2
    assert edited(cheb_too_big) == 6
    assert edited(chemact_on_elem) == 2
    assert edited(sri_bad) == 2
    assert edited(eff_on_plog) == 2
    assert _status(api, _write(tmp_path, good.replace(" SRI ", " SRI2 ", 1))) == 2


def test_noalloc_and_calibration_argument_checks(api, tmp_path):
    lib = api.library()
    assert lib.pj_batch_eval_noalloc(None, 1, 0, 0, None) == 1          # NULL batch
    b = ctypes.c_void_p()
    assert lib.pj_batch_create(ctypes.byref(b)) == 0
    assert lib.pj_batch_eval_noalloc(b, 2, 0, 0, None) == 1             # dense is not a batch mode
    assert lib.pj_batch_eval_noalloc(b, 1, 0, 0, None) == 0             # empty batch: nothing to do
    lib.pj_batch_free(b)
    dummy = ctypes.c_void_p(16)
    assert lib.pj_calibrate_fp64(4, 8, 1, dummy, dummy, None) == 1        # bad function
    assert lib.pj_calibrate_fp64(0, -1, 1, dummy, dummy, None) == 1       # negative size
    assert lib.pj_calibrate_fp64(0, 8, 0, dummy, dummy, None) == 1        # no repetition
    assert lib.pj_calibrate_fp64(0, 8, 1, None, dummy, None) == 1         # NULL input
    assert lib.pj_calibrate_fp64(0, 0, 1, None, None, None) == 0          # empty: nothing to do
