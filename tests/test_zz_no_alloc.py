"""The allocation-free batch entry point (pj_batch_eval_noalloc) against the
batch's persistent launch (pj_batch_eval), through the C-ABI: bit for bit at
one wave per workgroup (every addition in program order), and within the
parity gates of the oracle at the batch's default shape; two calls in a
row, the second on a smaller batch (fewer segments and states), and a batch
beyond the table's 64 segments is refused."""
import numpy as np
import pytest

import oracle
from oracle.gates import check_jac, check_source
from paper_1809_01029_amd import synth
from conftest import workload_file

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


def build(torch, api, mech_dir, segments, mode, layout, seed):
    b = api.Batch()
    segs = []
    for name, n in segments:
        m, path = workload_file(name, mech_dir)
        mech = api.load_mechanism(path)
        st = synth.make_states(m, n, seed + n)
        x, p = synth.pack_state(st, "conp", "C")
        v = np.random.default_rng(seed + n).standard_normal(x.shape)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a if layout == "C" else a.T)).cuda()
        xs, vs, ps = dev(x), dev(v), torch.from_numpy(p.copy()).cuda()
        d = torch.zeros_like(xs)
        if mode == "sparse":
            out = torch.zeros((mech.nnz, n) if layout == "F" else (n, mech.nnz), dtype=torch.float64, device="cuda")
        elif mode == "adjoint":
            out = torch.zeros_like(xs)
        else:
            out = None
        grad = torch.zeros((3, mech.n_reactions), dtype=torch.float64, device="cuda") if mode == "adjoint" else None
        b.add(mech, xs, ps, layout, out=out, dstate=d, v=vs if mode == "adjoint" else None, grad=grad)
        segs.append(dict(name=name, path=path, mech=mech, x=x, p=p, v=v, d=d, out=out, grad=grad))
    return b, segs


def outputs(segs):
    return [(s["d"].clone(), None if s["out"] is None else s["out"].clone(),
             None if s["grad"] is None else s["grad"].clone()) for s in segs]


def clear(segs):
    for s in segs:
        s["d"].fill_(float("nan"))
        if s["out"] is not None:
            s["out"].fill_(float("nan"))
        if s["grad"] is not None:
            s["grad"].fill_(7.0)


def host(t, layout):
    a = t.cpu().numpy()
    return a if layout == "C" else a.T


@pytest.mark.parametrize("mode,layout", [("source", "C"), ("sparse", "F"), ("sparse", "C"), ("adjoint", "C")])
def test_noalloc_matches_batch_launch(torch_cuda, api, mech_dir, mode, layout):
    torch = torch_cuda
    runs = [[("ns13", 300), ("ns53", 150), ("ns111", 60)], [("ns53", 40), ("ns13", 17)]]
    for k, segments in enumerate(runs):
        b, segs = build(torch, api, mech_dir, segments, mode, layout, 100 * k)
        b.set_strategy(mode, False)
        # one wave per workgroup: the two entry points give the same bits
        b.set_launch(mode, 2, 1)
        b.eval(mode, "conp", layout)
        torch.cuda.synchronize()
        ref = outputs(segs)
        clear(segs)
        b.eval_noalloc(mode, "conp", layout)
        torch.cuda.synchronize()
        note(f"noalloc {mode} {layout} call {k}: {len(segments)} segments")
        for s, (d0, o0, g0) in zip(segs, ref):
            assert torch.equal(s["d"], d0), (k, s["name"])
            if o0 is not None:
                assert torch.equal(s["out"], o0), (k, s["name"])
            if g0 is not None:
                # parameter sums: workgroups add them with device atomics
                torch.testing.assert_close(s["grad"], g0, rtol=1e-12, atol=1e-300)
        # the batch's default shape: inside the oracle's gates
        b.set_launch(mode, 0, 0)
        clear(segs)
        b.eval_noalloc(mode, "conp", layout)
        torch.cuda.synchronize()
        for s in segs:
            o = oracle.Oracle(s["path"])
            f_o, f_b = o.source(s["x"], s["p"], "conp", bound=True)
            check_source(host(s["d"], layout), f_o, f_b, f"noalloc {s['name']} source")
            if mode == "sparse":
                J_o, J_b = o.jacobian(s["x"], s["p"], "conp", bound=True)
                check_jac(api.sparse_to_dense(s["mech"], s["out"].cpu().numpy(), layout), J_o, J_b,
                          f"noalloc {s['name']} Jacobian")
            if mode == "adjoint":
                j_o, g_o, j_b, g_b = o.adjoint(s["x"], s["p"], s["v"], "conp", bound=True)
                check_jac(host(s["out"], layout), j_o, j_b, f"noalloc {s['name']} J^T v")
                check_jac(s["grad"].cpu().numpy(), g_o, g_b, f"noalloc {s['name']} parameter sums")


def test_noalloc_refuses_too_many_segments(torch_cuda, api, mech_dir):
    torch = torch_cuda
    m, path = workload_file("ns13", mech_dir)
    mech = api.load_mechanism(path)
    b = api.Batch()
    st = synth.make_states(m, 2, 5)
    x, p = synth.pack_state(st, "conp", "C")
    xs, ps = torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda()
    outs = [torch.empty_like(xs) for _ in range(65)]
    for d in outs:
        b.add(mech, xs, ps, "C", dstate=d)
    with pytest.raises(api.PjError) as ei:
        b.eval_noalloc("source", "conp", "C")
    assert "at most 64" in str(ei.value)
