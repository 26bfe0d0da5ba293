"""Parity of the HIP adjoint (pj_eval_adjoint) with the oracle's adjoint.

J^T v per state and the batch-summed Arrhenius-parameter derivatives are
compared element by element with the oracle on the same seeded inputs, under
the Jacobian gate of ``oracle.gates`` (1e-8 relative with a 1e-20 floor,
widened by the oracle's running error bound only where that bound is not
small against the value).  The differentiable wrapper is checked
against the same values and against central differences of the GPU source
terms.
"""
import copy

import numpy as np
import pytest

import oracle
from oracle.gates import check_jac, check_source
from paper_1809_01029_amd import synth
from conftest import TINY_SEEDS, tiny_file, workload_file

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


def note(*a):
    print(*a, flush=True)


def _dev(torch, a_c, layout):
    a = a_c if layout == "C" else np.ascontiguousarray(a_c.T)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t, layout):
    a = t.cpu().numpy()
    return a if layout == "C" else a.T


check = check_jac


def run(torch, api, path, x, p, v, form, layout):
    o = oracle.Oracle(path)
    mech = api.load_mechanism(path)
    note(f"adjoint {path} n={x.shape[0]} {form} {layout} shape {mech.launch_shape(3)}")
    xs, ps, vs = _dev(torch, x, layout), torch.from_numpy(p.copy()).cuda(), _dev(torch, v, layout)
    d = torch.empty_like(xs)
    jtv, grad = api.eval_adjoint(mech, xs, ps, vs, form, layout, dstate=d)
    torch.cuda.synchronize()
    j_o, g_o, j_s, g_s = o.adjoint(x, p, v, form, bound=True)
    check(_host(jtv, layout), j_o, j_s, "J^T v")
    check(grad.cpu().numpy(), g_o, g_s, "parameter derivatives")
    f_o, f_s = o.source(x, p, form, bound=True)
    check_source(_host(d, layout), f_o, f_s, "fused source terms")
    return mech


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("seed", TINY_SEEDS)
@pytest.mark.parametrize("bath", [False, True])
def test_adjoint_tiny(torch_cuda, api, seed, bath, form, layout, mech_dir):
    kw = dict(bath_reactions=1, bath_efficiency=True) if bath else {}
    m, path = tiny_file(seed, mech_dir, **kw)
    st = synth.make_states(m, 29, 300 + seed)
    x, p = synth.pack_state(st, form, "C")
    v = np.random.default_rng(seed).standard_normal(x.shape)
    run(torch_cuda, api, path, x, p, v, form, layout)


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form", ["conp", "conv"])
@pytest.mark.parametrize("name,n", [("ns13", 1024), ("ns53", 150), ("ns111", 40), ("ns360", 4)])
def test_adjoint_workloads(torch_cuda, api, name, n, form, layout, mech_dir):
    m, path = workload_file(name, mech_dir)
    w = synth.WORKLOADS[name]
    st = synth.make_states(m, n, w.state_seed + 3, T_range=w.T_range, P_range_atm=w.P_range_atm)
    x, p = synth.pack_state(st, form, "C")
    v = np.random.default_rng(7).standard_normal(x.shape)
    run(torch_cuda, api, path, x, p, v, form, layout)


def test_adjoint_shapes_and_edges(torch_cuda, api, mech_dir):
    torch = torch_cuda
    m, path = workload_file("ns53", mech_dir)
    o = oracle.Oracle(path)
    mech = api.load_mechanism(path)
    for S, w in [(1, 1), (1, 4), (2, 2), (4, 1), (4, 8)]:
        mech.set_launch(S, w)
        for n in (1, 2, 65, 333):
            st = synth.make_states(m, n, 900 + n)
            x, p = synth.pack_state(st, "conv", "C")
            v = np.random.default_rng(n).standard_normal(x.shape)
            note(f"adjoint shape {mech.launch_shape(3)} n={n}")
            xs, ps, vs = _dev(torch, x, "C"), torch.from_numpy(p).cuda(), _dev(torch, v, "C")
            jtv, grad = api.eval_adjoint(mech, xs, ps, vs, "conv", "C")
            torch.cuda.synchronize()
            j_o, g_o, j_s, g_s = o.adjoint(x, p, v, "conv", bound=True)
            check(jtv.cpu().numpy(), j_o, j_s, f"J^T v S={S} w={w} n={n}")
            check(grad.cpu().numpy(), g_o, g_s, f"gradient S={S} w={w} n={n}")
    # an empty batch: no work, gradient sums are zero
    e = torch.empty((0, mech.N), dtype=torch.float64, device="cuda")
    grad = torch.full((3, mech.n_reactions), 7.0, dtype=torch.float64, device="cuda")
    api.eval_adjoint(mech, e, torch.empty(0, dtype=torch.float64, device="cuda"), e, "conp", "C", grad=grad)
    torch.cuda.synchronize()
    assert torch.count_nonzero(grad).item() == 0


def test_set_arrhenius_and_autograd(torch_cuda, api, mech_dir):
    torch = torch_cuda
    m, path = workload_file("ns53", mech_dir)
    mech = api.load_mechanism(path)
    lnA0, b0, t0 = mech.arrhenius()
    np.testing.assert_array_equal(lnA0, [r.lnA for r in m.reactions])
    rng = np.random.default_rng(5)
    lnA = lnA0 + 0.3 * rng.standard_normal(lnA0.shape)
    b = b0 + 0.05 * rng.standard_normal(b0.shape)
    th = t0 * (1 + 0.02 * rng.standard_normal(t0.shape))
    # the oracle reads the same parameters from a rewritten description
    m2 = copy.deepcopy(m)
    for i, r in enumerate(m2.reactions):
        r.lnA, r.b, r.theta = float(lnA[i]), float(b[i]), float(th[i])
    p2 = path + ".recalibrated.pjm"
    synth.write_mechanism(m2, p2)
    o = oracle.Oracle(p2)
    st = synth.make_states(m, 64, 4242)
    x, p = synth.pack_state(st, "conp", "C")
    wv = rng.standard_normal(x.shape)
    xs = torch.from_numpy(x).cuda().requires_grad_(True)
    ps = torch.from_numpy(p).cuda()
    tl = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (lnA, b, th)]
    f = api.source_terms(mech, xs, ps, *tl, "conp", "C")
    # the call carries its parameters: the mechanism's tables are untouched
    np.testing.assert_array_equal(mech.arrhenius()[0], lnA0)
    f_o, f_s = o.source(x, p, "conp", bound=True)
    check_source(f.detach().cpu().numpy(), f_o, f_s, "autograd source terms")
    loss = (f * torch.from_numpy(wv).cuda()).sum()
    loss.backward()
    j_o, g_o, j_s, g_s = o.adjoint(x, p, wv, "conp", bound=True)
    check(xs.grad.cpu().numpy(), j_o, j_s, "autograd state gradient")
    for a in range(3):
        check(tl[a].grad.cpu().numpy(), g_o[a], g_s[a], f"autograd parameter {a}")
    # central differences of the GPU source terms along a random direction
    u = rng.standard_normal(x.shape) * np.abs(x)
    h = 1e-6
    arr = torch.stack([t.detach() for t in tl]).contiguous()
    with torch.no_grad():
        fp = api.eval_source(mech, torch.from_numpy(x + h * u).cuda(), ps, "conp", "C", arrhenius=arr).cpu().numpy()
        fm = api.eval_source(mech, torch.from_numpy(x - h * u).cuda(), ps, "conp", "C", arrhenius=arr).cpu().numpy()
    fd = np.sum(wv * (fp - fm) / (2 * h), axis=1)
    ad = np.sum(u * xs.grad.cpu().numpy(), axis=1)
    np.testing.assert_allclose(ad, fd, rtol=1e-5, atol=1e-6 * np.abs(ad).max())
    # the same parameters installed in the mechanism's tables
    mech.set_arrhenius(lnA, b, th)
    np.testing.assert_array_equal(mech.arrhenius()[0], lnA)
    with torch.no_grad():
        f2 = api.eval_source(mech, torch.from_numpy(x).cuda(), ps, "conp", "C").cpu().numpy()
    check_source(f2, f_o, f_s, "source terms after set_arrhenius")
    mech.set_arrhenius(lnA0, b0, t0)


def test_autograd_two_parameter_sets(torch_cuda, api, mech_dir):
    """Two forward passes with different Arrhenius parameters before either
    backward pass: each graph's gradient is the oracle's at its own
    parameters (the parameters travel with the call, not with the
    mechanism)."""
    torch = torch_cuda
    m, path = workload_file("ns53", mech_dir)
    mech = api.load_mechanism(path)
    lnA0, b0, t0 = mech.arrhenius()
    rng = np.random.default_rng(12)
    st = synth.make_states(m, 96, 777)
    x, p = synth.pack_state(st, "conv", "F")
    xc, _ = synth.pack_state(st, "conv", "C")
    ps = torch.from_numpy(p).cuda()
    sets, runs = [], []
    for k in range(2):
        lnA = lnA0 + 0.2 * rng.standard_normal(lnA0.shape)
        b = b0 + 0.05 * rng.standard_normal(b0.shape)
        th = t0 * (1 + 0.02 * rng.standard_normal(t0.shape))
        m2 = copy.deepcopy(m)
        for i, r in enumerate(m2.reactions):
            r.lnA, r.b, r.theta = float(lnA[i]), float(b[i]), float(th[i])
        p2 = f"{path}.set{k}.pjm"
        synth.write_mechanism(m2, p2)
        xs = torch.from_numpy(np.ascontiguousarray(x)).cuda().requires_grad_(True)
        tl = [torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True) for a in (lnA, b, th)]
        f = api.source_terms(mech, xs, ps, *tl, "conv", "F")
        wv = rng.standard_normal(xc.shape)
        sets.append((p2, wv))
        runs.append((f, xs, tl))
    # backward of the first graph after the second forward, then the second
    for k in (0, 1):
        f, xs, tl = runs[k]
        p2, wv = sets[k]
        note(f"two parameter sets: backward {k}")
        (f * torch.from_numpy(np.ascontiguousarray(wv.T)).cuda()).sum().backward()
        o = oracle.Oracle(p2)
        f_o, f_s = o.source(xc, p, "conv", bound=True)
        check_source(f.detach().cpu().numpy().T, f_o, f_s, f"forward {k}")
        j_o, g_o, j_s, g_s = o.adjoint(xc, p, wv, "conv", bound=True)
        check(xs.grad.cpu().numpy().T, j_o, j_s, f"state gradient {k}")
        for a in range(3):
            check(tl[a].grad.cpu().numpy(), g_o[a], g_s[a], f"parameter gradient {k}.{a}")
    np.testing.assert_array_equal(mech.arrhenius()[0], lnA0)


def test_adjoint_full_size_sampled(torch_cuda, api, mech_dir):
    """111 species at 262,144 states: J^T v on sampled states against the
    oracle, and the batch sums equal the sum over two halves of the batch."""
    torch = torch_cuda
    m, path = workload_file("ns111", mech_dir)
    w = synth.WORKLOADS["ns111"]
    n = w.n_states
    st = synth.make_states(m, n, w.state_seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
    x, p = synth.pack_state(st, "conp", "C")
    v = np.random.default_rng(8).standard_normal(x.shape)
    mech = api.load_mechanism(path)
    xs, ps, vs = torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(v).cuda()
    note("adjoint full size 262144")
    jtv, grad = api.eval_adjoint(mech, xs, ps, vs, "conp", "C")
    h = n // 2
    _, g1 = api.eval_adjoint(mech, xs[:h].contiguous(), ps[:h].contiguous(), vs[:h].contiguous(), "conp", "C")
    _, g2 = api.eval_adjoint(mech, xs[h:].contiguous(), ps[h:].contiguous(), vs[h:].contiguous(), "conp", "C")
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(3).choice(n, 24, replace=False))
    j_o, _, j_s, _ = oracle.Oracle(path).adjoint(x[idx], p[idx], v[idx], "conp", bound=True)
    check(jtv.cpu().numpy()[idx], j_o, j_s, "full-size J^T v sample")
    g, gs = grad.cpu().numpy(), (g1 + g2).cpu().numpy()
    np.testing.assert_allclose(g, gs, rtol=1e-9, atol=1e-12 * np.abs(g).max())
    assert torch.isfinite(jtv).all()


def test_adjoint_autotune(torch_cuda, api, mech_dir):
    torch = torch_cuda
    m, path = workload_file("ns53", mech_dir)
    st = synth.make_states(m, 1500, 61)
    x, p = synth.pack_state(st, "conv", "C")
    v = np.random.default_rng(4).standard_normal(x.shape)
    mech = api.load_mechanism(path)
    xs, ps, vs = torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(v).cuda()
    S, W, ms = api.autotune(mech, xs, ps, "conv", "C", mode="adjoint", reps=1)
    note(f"adjoint autotune: S={S} W={W} {ms:.4f} ms")
    assert mech.launch_shape(3) == (S, W) and S in (1, 2, 4) and 1 <= W <= 8
    jtv, grad = api.eval_adjoint(mech, xs, ps, vs, "conv", "C")
    torch.cuda.synchronize()
    j_o, g_o, j_s, g_s = oracle.Oracle(path).adjoint(x, p, v, "conv", bound=True)
    check(jtv.cpu().numpy(), j_o, j_s, "tuned J^T v")
    check(grad.cpu().numpy(), g_o, g_s, "tuned parameter derivatives")
