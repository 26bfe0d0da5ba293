"""Ragged multi-mechanism batches (pj_batch_*): one launch over segments of
states of different mechanisms, and its captured HIP graph.

Every segment's outputs are checked against the oracle under the same gates
as the per-mechanism calls; with one wave per workgroup the batch reproduces
the per-mechanism launch of the same shape bit for bit; graph replays, with
eager work and synchronisation between them, reproduce the eager batch.
"""
import numpy as np
import pytest

import oracle
from oracle.gates import check_jac, check_source
from paper_1809_01029_amd import synth
from conftest import workload_file

pytestmark = pytest.mark.gpu

SEGMENTS = [("ns13", 300), ("ns53", 150), ("empty", 0), ("ns111", 60)]


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


def build(torch, api, mech_dir, form, layout, mode):
    segs = []
    b = api.Batch()
    for name, n in SEGMENTS:
        nm = "ns13" if name == "empty" else name
        m, path = workload_file(nm, mech_dir)
        mech = api.load_mechanism(path)
        st = synth.make_states(m, n, 500 + n)
        x, p = synth.pack_state(st, form, "C")
        v = np.random.default_rng(n).standard_normal(x.shape)
        xs, ps, vs = _dev(torch, x, layout), torch.from_numpy(p.copy()).cuda(), _dev(torch, v, layout)
        d = torch.zeros_like(xs)
        if mode == "sparse":
            out = torch.zeros((mech.nnz, n) if layout == "F" else (n, mech.nnz), dtype=torch.float64, device="cuda")
        elif mode == "adjoint":
            out = torch.zeros_like(xs)
        else:
            out = None
        grad = torch.zeros((3, mech.n_reactions), dtype=torch.float64, device="cuda") if mode == "adjoint" else None
        b.add(mech, xs, ps, layout, out=out, dstate=d, v=vs if mode == "adjoint" else None, grad=grad)
        segs.append(dict(name=nm, path=path, mech=mech, x=x, p=p, v=v, xs=xs, ps=ps, vs=vs, d=d, out=out, grad=grad))
    return b, segs


def check_against_oracle(api, segs, form, layout, mode):
    for sg in segs:
        if sg["x"].shape[0] == 0:
            continue
        o = oracle.Oracle(sg["path"])
        x, p = sg["x"], sg["p"]
        f_o, f_s = o.source(x, p, form, bound=True)
        check_source(_host(sg["d"], layout), f_o, f_s, f"{sg['name']} source terms")
        if mode == "sparse":
            J_o, J_s = o.jacobian(x, p, form, bound=True)
            Jg = api.sparse_to_dense(sg["mech"], sg["out"].cpu().numpy(), layout)
            check_jac(Jg, J_o, J_s, f"{sg['name']} Jacobian")
        if mode == "adjoint":
            j_o, g_o, j_s, g_s = o.adjoint(x, p, sg["v"], form, bound=True)
            check_jac(_host(sg["out"], layout), j_o, j_s, f"{sg['name']} J^T v")
            check_jac(sg["grad"].cpu().numpy(), g_o, g_s, f"{sg['name']} grad")


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form,mode", [("conp", "source"), ("conp", "sparse"), ("conv", "sparse"),
                                       ("conp", "adjoint"), ("conv", "adjoint")])
def test_batch_matches_oracle(torch_cuda, api, form, mode, layout, mech_dir):
    torch = torch_cuda
    b, segs = build(torch, api, mech_dir, form, layout, mode)
    note(f"batch {form} {mode} {layout} shape {b.launch_shape(mode)}")
    b.eval(mode, form, layout)
    torch.cuda.synchronize()
    check_against_oracle(api, segs, form, layout, mode)


@pytest.mark.parametrize("mode", ["source", "sparse"])
def test_batch_equals_per_mechanism_launch(torch_cuda, api, mode, mech_dir):
    """One wave per workgroup: every accumulation in program order, so the
    batch gives the bits of the per-mechanism launch at each segment's own
    states per workgroup (the smaller mechanisms take more states in the LDS
    the largest one sets)."""
    torch = torch_cuda
    b, segs = build(torch, api, mech_dir, "conp", "C", mode)
    for S in (1, 2, 4):
        b.set_launch(mode, S, 1)
        seg_S = b.segment_states(mode)
        note(f"{mode} base S={S}: segment states {seg_S}")
        assert all(s >= S and s <= 16 and (s & (s - 1)) == 0 for s in seg_S)
        # the largest mechanism keeps the base shape
        assert seg_S[-1] == S
        if S == 1:
            assert seg_S[0] > seg_S[-1]   # the 13-species segment holds more states
        b.eval(mode, "conp", "C")
        for k, sg in enumerate(segs):
            if sg["x"].shape[0] == 0:
                continue
            sg["mech"].set_launch(seg_S[k], 1)
            if mode == "source":
                ref = api.eval_source(sg["mech"], sg["xs"], sg["ps"], "conp", "C")
                torch.cuda.synchronize()
                assert torch.equal(ref, sg["d"]), sg["name"]
            else:
                dref = torch.empty_like(sg["xs"])
                ref = api.eval_jacobian_sparse(sg["mech"], sg["xs"], sg["ps"], "conp", "C", dstate=dref)
                torch.cuda.synchronize()
                assert torch.equal(ref, sg["out"]) and torch.equal(dref, sg["d"]), sg["name"]


@pytest.mark.parametrize("per_segment", [False, True])
@pytest.mark.parametrize("mode", ["sparse", "adjoint"])
def test_batch_graph_replays(torch_cuda, api, mode, per_segment, mech_dir):
    torch = torch_cuda
    b, segs = build(torch, api, mech_dir, "conp", "F", mode)
    b.set_launch(mode, 2, 1)
    b.set_strategy(mode, per_segment)
    if per_segment:
        # one wave per workgroup for every mechanism too: replays then give
        # the eager run's bits
        for sg in segs:
            sg["mech"].set_launch(2, 1)
    b.eval(mode, "conp", "F")
    torch.cuda.synchronize()
    ref = [(sg["d"].clone(), None if sg["out"] is None else sg["out"].clone(),
            None if sg["grad"] is None else sg["grad"].clone()) for sg in segs]
    for r in range(3):
        # eager work and a synchronisation between replays
        for sg in segs:
            sg["d"].zero_()
            if sg["out"] is not None:
                sg["out"].fill_(float("nan"))
            if sg["grad"] is not None:
                sg["grad"].fill_(3.0)
        api.eval_source(segs[0]["mech"], segs[0]["xs"], segs[0]["ps"], "conp", "F")
        torch.cuda.synchronize()
        b.eval(mode, "conp", "F", graph=True)
        torch.cuda.synchronize()
        note(f"graph replay {r}")
        for sg, (d0, o0, g0) in zip(segs, ref):
            assert torch.equal(sg["d"], d0), (r, sg["name"])
            if o0 is not None:
                assert torch.equal(sg["out"], o0), (r, sg["name"])
            if g0 is not None:
                # parameter sums are added with device atomics: equal to rounding
                torch.testing.assert_close(sg["grad"], g0, rtol=1e-12, atol=1e-300)
    check_against_oracle(api, segs, "conp", "F", mode)


def test_batch_autotune(torch_cuda, api, mech_dir):
    torch = torch_cuda
    b, segs = build(torch, api, mech_dir, "conp", "C", "sparse")
    S, W, ms = b.autotune("sparse", "conp", "C", reps=1)
    note(f"batch autotune: S={S} W={W} {ms:.4f} ms")
    if S == 0:
        # one launch per segment won; the best persistent shape is kept
        assert W == 0 and b.strategy("sparse")
        Sp, Wp = b.launch_shape("sparse")
        assert Sp in (1, 2, 4, 8, 16) and 1 <= Wp <= 8
    else:
        assert not b.strategy("sparse")
        assert b.launch_shape("sparse") == (S, W) and S in (1, 2, 4, 8, 16) and 1 <= W <= 8
    for sg in segs:
        if sg["out"] is not None:
            sg["out"].zero_()
    b.eval("sparse", "conp", "C")
    torch.cuda.synchronize()
    check_against_oracle(api, segs, "conp", "C", "sparse")


@pytest.mark.parametrize("layout", ["F", "C"])
@pytest.mark.parametrize("form,mode", [("conp", "source"), ("conv", "sparse"), ("conp", "adjoint")])
def test_batch_per_segment_launches(torch_cuda, api, form, mode, layout, mech_dir):
    """One launch per segment at each mechanism's own shape: the oracle's
    values, and (one wave per workgroup) the single-mechanism calls' bits."""
    torch = torch_cuda
    b, segs = build(torch, api, mech_dir, form, layout, mode)
    for k, sg in enumerate(segs):
        sg["mech"].set_launch((1, 2, 4)[k % 3], 1)
    b.set_strategy(mode, True)
    assert b.strategy(mode)
    note(f"batch per segment {form} {mode} {layout}")
    b.eval(mode, form, layout)
    torch.cuda.synchronize()
    check_against_oracle(api, segs, form, layout, mode)
    if mode == "adjoint":
        return
    for sg in segs:
        if sg["x"].shape[0] == 0:
            continue
        if mode == "source":
            ref = api.eval_source(sg["mech"], sg["xs"], sg["ps"], form, layout)
            torch.cuda.synchronize()
            assert torch.equal(ref, sg["d"]), sg["name"]
        else:
            dref = torch.empty_like(sg["xs"])
            ref = api.eval_jacobian_sparse(sg["mech"], sg["xs"], sg["ps"], form, layout, dstate=dref)
            torch.cuda.synchronize()
            assert torch.equal(ref, sg["out"]) and torch.equal(dref, sg["d"]), sg["name"]


# The ragged configuration at its stated size: 3,000 / 70,000 / 20,000 states
# of the 13-, 53- and 111-species mechanisms (state seeds 2013, 2053, 2111),
# v ~ N(0, 1) with seed 7.
C5 = [("ns13", 3000, 2013), ("ns53", 70000, 2053), ("ns111", 20000, 2111)]


@pytest.mark.parametrize("strategy", ["auto", "persistent"])
@pytest.mark.parametrize("mode", ["source", "adjoint"])
def test_ragged_batch_full_counts(torch_cuda, api, mode, strategy, mech_dir):
    """The ragged batch at its stated counts through the captured graph
    (autotuned strategy), replayed twice: every segment sampled (first and
    last state included) against the oracle; for the adjoint, each
    segment's batch-summed parameter derivatives equal the sum of two
    per-mechanism calls over the two halves of its states, and on 64 sampled
    states they match the oracle's and central differences of the GPU source
    terms (step 1e-6 relative)."""
    torch = torch_cuda
    b = api.Batch()
    segs = []
    rng_v = np.random.default_rng(7)
    for name, n, seed in C5:
        m, path = workload_file(name, mech_dir)
        w = synth.WORKLOADS[name]
        mech = api.load_mechanism(path)
        st = synth.make_states(m, n, seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
        x, p = synth.pack_state(st, "conp", "C")
        v = rng_v.standard_normal(x.shape)
        xs, ps, vs = torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(v).cuda()
        d = torch.zeros_like(xs)
        out = torch.zeros_like(xs) if mode == "adjoint" else None
        grad = torch.zeros((3, mech.n_reactions), dtype=torch.float64, device="cuda") if mode == "adjoint" else None
        b.add(mech, xs, ps, "C", out=out, dstate=d, v=vs if mode == "adjoint" else None, grad=grad)
        segs.append(dict(name=name, path=path, mech=mech, x=x, p=p, v=v, xs=xs, ps=ps, vs=vs, d=d, out=out,
                         grad=grad, n=n))
    S, W, ms = b.autotune(mode, "conp", "C", reps=1)
    if strategy == "persistent":
        # the one persistent launch at its best shape, whatever won
        b.set_strategy(mode, False)
    note(f"ragged {mode} at full counts: autotune S={S} W={W} per_segment={b.strategy(mode)} {ms:.3f} ms, "
         f"shape {b.launch_shape(mode)}, segment states {b.segment_states(mode)}")
    for r in range(2):
        for sg in segs:
            sg["d"].zero_()
            if sg["out"] is not None:
                sg["out"].fill_(float("nan"))
        b.eval(mode, "conp", "C", graph=True)
        torch.cuda.synchronize()
        note(f"ragged {mode} graph replay {r}")
    for sg in segs:
        n = sg["n"]
        rng = np.random.default_rng(sg["n"])
        idx = np.sort(np.concatenate([rng.choice(n, 30, replace=False), [0, n - 1]]))
        o = oracle.Oracle(sg["path"])
        x, p, v = sg["x"][idx], sg["p"][idx], sg["v"][idx]
        f_o, f_s = o.source(x, p, "conp", bound=True)
        check_source(sg["d"].cpu().numpy()[idx], f_o, f_s, f"{sg['name']} source terms (sample)")
        if mode != "adjoint":
            continue
        j_o, _, j_s, _ = o.adjoint(x, p, v, "conp", bound=True)
        check_jac(sg["out"].cpu().numpy()[idx], j_o, j_s, f"{sg['name']} J^T v (sample)")
        # batch sums = the sum over two halves, each by a per-mechanism call
        h = n // 2
        _, g1 = api.eval_adjoint(sg["mech"], sg["xs"][:h].contiguous(), sg["ps"][:h].contiguous(),
                                 sg["vs"][:h].contiguous(), "conp", "C")
        _, g2 = api.eval_adjoint(sg["mech"], sg["xs"][h:].contiguous(), sg["ps"][h:].contiguous(),
                                 sg["vs"][h:].contiguous(), "conp", "C")
        g, gs = sg["grad"].cpu().numpy(), (g1 + g2).cpu().numpy()
        np.testing.assert_allclose(g, gs, rtol=1e-9, atol=1e-12 * np.abs(g).max())
        # 64 sampled states: the oracle's batch sums and central differences
        i64 = np.sort(rng.choice(n, 64, replace=False))
        x, p, v = sg["x"][i64], sg["p"][i64], sg["v"][i64]
        xs, ps, vs = torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda(), torch.from_numpy(v).cuda()
        _, g64 = api.eval_adjoint(sg["mech"], xs, ps, vs, "conp", "C")
        _, g_o, _, g_s = o.adjoint(x, p, v, "conp", bound=True)
        check_jac(g64.cpu().numpy(), g_o, g_s, f"{sg['name']} parameter sums (64 states)")
        arr = torch.from_numpy(np.stack(sg["mech"].arrhenius())).cuda()
        g64 = g64.cpu().numpy()
        for a in range(3):
            for i in rng.choice(sg["mech"].n_reactions, 8, replace=False):
                base = float(arr[a, i])
                h_ = 1e-6 * max(abs(base), 1.0)
                vals = []
                for sgn in (1.0, -1.0):
                    ar = arr.clone()
                    ar[a, i] = base + sgn * h_
                    f = api.eval_source(sg["mech"], xs, ps, "conp", "C", arrhenius=ar)
                    vals.append(float(torch.sum(f * vs)))
                fd = (vals[0] - vals[1]) / (2 * h_)
                scale = np.abs(g64[a]).max()
                assert abs(fd - g64[a, i]) <= 1e-5 * abs(g64[a, i]) + 1e-7 * scale, \
                    (sg["name"], a, int(i), fd, g64[a, i])
