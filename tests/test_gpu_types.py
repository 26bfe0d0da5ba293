"""Parity of the HIP path with the oracle on mechanisms that hold every
reaction type the library supports: SRI falloff, chemically activated
(Lindemann, Troe, SRI forms), P-Log and Chebyshev rate constants, besides
elementary, third-body, Lindemann and Troe reactions.

Same gates as the other parity tests (``oracle.gates``: source terms 1e-10
relative, Jacobian and adjoint 1e-8 relative with a 1e-20 floor, widened by
the oracle's running error bound only on cancelling entries), on all states of
tiny mechanisms and on sampled states of the 111-species all-types workload,
in both forms and layouts, at several launch shapes, in the adjoint, in a
ragged batch and in the approximate-Jacobian variant.
"""
import numpy as np
import pytest

import oracle
from paper_1809_01029_amd import synth
from conftest import TYPES_SEEDS, types_file, workload_file
from test_gpu_parity import check_jac, check_source, note, run_case, src_to_c

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def api(torch_cuda):
    from paper_1809_01029_amd import api as a
    return a


def _dev(torch, a_c, layout):
    a = a_c if layout == "C" else np.ascontiguousarray(a_c.T)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t, layout):
    a = t.cpu().numpy()
    return a if layout == "C" else a.T


def _wide_pressures(m, n, seed, form):
    # pressures from 0.05 to 300 atm, so that P-Log reactions see both ends of
    # their tables and Chebyshev fits are evaluated slightly outside theirs
    st = synth.make_states(m, n, seed, P_range_atm=(0.05, 300.0))
    return synth.pack_state(st, form, "C")


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TYPES_SEEDS)
@pytest.mark.parametrize("bath", [False, True])
def test_types_tiny(torch_cuda, api, seed, bath, form, layout, mech_dir):
    m, path = types_file(seed, mech_dir, bath=bath)
    x, p = _wide_pressures(m, 41, 200 + seed, form)
    run_case(torch_cuda, api, path, x, p, form, layout)


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form", ["conp", "conv"])
def test_types_workload_sampled(torch_cuda, api, form, layout, mech_dir):
    # 111 species with every type, 2,000 states (a ragged last group), the
    # oracle on 40 sampled states
    m, path = workload_file("ns111x", mech_dir)
    w = synth.WORKLOADS["ns111x"]
    st = synth.make_states(m, 2000, w.state_seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
    x, p = synth.pack_state(st, form, "C")
    sample = np.random.default_rng(3).choice(2000, 40, replace=False)
    sample[0] = 1999
    run_case(torch_cuda, api, path, x, p, form, layout, dense=True, sample=sample)


@pytest.mark.parametrize("layout", ["F", "C"])
def test_types_launch_shapes(torch_cuda, api, layout, mech_dir):
    torch = torch_cuda
    m, path = types_file(TYPES_SEEDS[1], mech_dir, bath=True)
    o = oracle.Oracle(path)
    for form in ("conp", "conv"):
        xc, pc = _wide_pressures(m, 133, 9, form)
        f_o, f_s = o.source(xc, pc, form, bound=True)
        J_o, J_s = o.jacobian(xc, pc, form, bound=True)
        mech = api.load_mechanism(path)
        xs, ps = _dev(torch, xc, layout), torch.from_numpy(pc.copy()).cuda()
        for S, wv in [(1, 1), (2, 4), (4, 2), (16, 1), (64, 1)]:
            mech.set_launch(S, wv)
            note(f"types launch S={S} waves={wv} {form} {layout} -> {mech.launch_shape(1)}")
            d = torch.empty_like(xs)
            j = api.eval_jacobian_sparse(mech, xs, ps, form, layout, dstate=d)
            torch.cuda.synchronize()
            check_source(src_to_c(d, layout), f_o, f_s, f"S={S} w={wv} source")
            check_jac(api.sparse_to_dense(mech, j.cpu().numpy(), layout), J_o, J_s, f"S={S} w={wv}")


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TYPES_SEEDS[:3])
def test_types_adjoint(torch_cuda, api, seed, form, layout, mech_dir):
    torch = torch_cuda
    m, path = types_file(seed, mech_dir, bath=True)
    x, p = _wide_pressures(m, 37, 400 + seed, form)
    v = np.random.default_rng(seed).standard_normal(x.shape)
    o = oracle.Oracle(path)
    mech = api.load_mechanism(path)
    note(f"types adjoint {path} {form} {layout}")
    xs, ps, vs = _dev(torch, x, layout), torch.from_numpy(p.copy()).cuda(), _dev(torch, v, layout)
    jtv, grad = api.eval_adjoint(mech, xs, ps, vs, form, layout)
    torch.cuda.synchronize()
    j_o, g_o, j_s, g_s = o.adjoint(x, p, v, form, bound=True)
    check_jac(_host(jtv, layout), j_o, j_s, "J^T v")
    check_jac(grad.cpu().numpy(), g_o, g_s, "parameter derivatives")


@pytest.mark.parametrize("form", ["conp", "conv"])
def test_types_approximate_jacobian(torch_cuda, api, form, mech_dir):
    torch = torch_cuda
    m, path = types_file(TYPES_SEEDS[2], mech_dir, bath=True)
    x, p = _wide_pressures(m, 50, 17, form)
    o = oracle.Oracle(path)
    mech = api.load_mechanism(path, options=api.OPT_APPROX_JACOBIAN)
    note(f"types approximate {path} {form}")
    xs, ps = _dev(torch, x, "C"), torch.from_numpy(p.copy()).cuda()
    j = api.eval_jacobian_sparse(mech, xs, ps, form, "C")
    torch.cuda.synchronize()
    J_o, J_s = o.jacobian(x, p, form, bound=True, approx=True)
    check_jac(api.sparse_to_dense(mech, j.cpu().numpy(), "C"), J_o, J_s, "approximate")


@pytest.mark.parametrize("mode", ["source", "sparse", "adjoint"])
def test_types_in_ragged_batch(torch_cuda, api, mode, mech_dir):
    torch = torch_cuda
    form, layout = "conv", "F"
    b = api.Batch()
    segs = []
    for k, (fn, n) in enumerate([(lambda: workload_file("ns13", mech_dir), 90),
                                 (lambda: types_file(TYPES_SEEDS[3], mech_dir, bath=True), 57),
                                 (lambda: workload_file("ns111x", mech_dir), 20)]):
        m, path = fn()
        mech = api.load_mechanism(path)
        x, p = _wide_pressures(m, n, 600 + k, form)
        v = np.random.default_rng(k).standard_normal(x.shape)
        xs, ps, vs = _dev(torch, x, layout), torch.from_numpy(p.copy()).cuda(), _dev(torch, v, layout)
        d = torch.zeros_like(xs)
        out = (torch.zeros((mech.nnz, n), dtype=torch.float64, device="cuda") if mode == "sparse"
               else torch.zeros_like(xs) if mode == "adjoint" else None)
        grad = torch.zeros((3, mech.n_reactions), dtype=torch.float64, device="cuda") if mode == "adjoint" else None
        b.add(mech, xs, ps, layout, out=out, dstate=d, v=vs if mode == "adjoint" else None, grad=grad)
        segs.append((path, mech, x, p, v, d, out, grad))
    note(f"types batch {mode}")
    b.eval(mode, form, layout)
    torch.cuda.synchronize()
    for path, mech, x, p, v, d, out, grad in segs:
        o = oracle.Oracle(path)
        f_o, f_s = o.source(x, p, form, bound=True)
        check_source(_host(d, layout), f_o, f_s, f"batch {path} source")
        if mode == "sparse":
            J_o, J_s = o.jacobian(x, p, form, bound=True)
            check_jac(api.sparse_to_dense(mech, out.cpu().numpy(), layout), J_o, J_s, f"batch {path}")
        if mode == "adjoint":
            j_o, g_o, j_s, g_s = o.adjoint(x, p, v, form, bound=True)
            check_jac(_host(out, layout), j_o, j_s, f"batch {path} J^T v")
            check_jac(grad.cpu().numpy(), g_o, g_s, f"batch {path} grad")
    b.close()


# random mechanisms holding every type: (seed, species, reactions); odd seeds
# let the bath gas react and give it an efficiency
RANDOM_TYPES = [(100, 11, 23), (101, 12, 30), (103, 14, 44), (104, 15, 51), (105, 16, 58),
                (106, 17, 24), (107, 18, 31), (108, 19, 38), (109, 20, 45), (112, 12, 25)]


@pytest.mark.parametrize("seed,ns,nr", RANDOM_TYPES)
def test_types_random_mechanisms(torch_cuda, api, seed, ns, nr, mech_dir):
    """Both forms and layouts at a launch shape drawn per mechanism, states
    from 500 to 2,500 K and 0.02 to 500 atm, a ragged last group."""
    from conftest import TYPES_MIX
    import os
    m = synth.make_mechanism(ns, nr, seed, mix=TYPES_MIX, zipf=0.5, bath_reactions=seed % 2,
                             bath_efficiency=bool(seed % 2))
    path = os.path.join(str(mech_dir), f"rtypes_{seed}.pjm")
    synth.write_mechanism(m, path)
    rng = np.random.default_rng(seed)
    S, W = [(1, 1), (1, 2), (2, 2), (2, 4), (4, 1), (4, 4), (8, 1), (16, 1)][seed % 8]
    st = synth.make_states(m, 77, seed, T_range=(500.0, 2500.0), P_range_atm=(0.02, 500.0))
    for form in ("conp", "conv"):
        x, p = synth.pack_state(st, form, "C")
        layout = "CF"[int(rng.integers(2))]
        run_case(torch_cuda, api, path, x, p, form, layout, dense=True)
        note(f"random types {seed} {form} at {S}x{W}")
        run_case(torch_cuda, api, path, x, p, form, "F" if layout == "C" else "C", dense=False, launch=(S, W))
