#!/usr/bin/env python3
"""Benchmark: states/s for thermochemical source terms + sparse Jacobian (FP64).

One step is one fused pass of the whole hot path (bath-gas closure, species
thermodynamics, rate constants, pressure modification, equilibrium constants,
rates of progress, production rates, source terms, analytical Jacobian on the
CSR pattern) over one batch of synthetic states already resident in HBM.  The
default workload is the 111-species / 784-reaction synthetic mechanism at
262,144 states, constant pressure, layout C (each state's values contiguous).

Prints ONE JSON line on stdout; progress goes to stderr.

``--copy-calibration`` instead runs a plain device copy of known size, the
reference that scales the rocprofv3 FETCH_SIZE / WRITE_SIZE readings into
bytes.
"""
import argparse
import concurrent.futures
import hashlib
import json
import platform
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "states/sec for source terms and sparse Jacobian (FP64, % of roofline)"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that decide the kernel's memory traffic; a traffic figure measured
# with other versions of them is not reported.
KERNEL_SOURCES = ["paper_1809_01029_amd/csrc/kernel_body.h", "paper_1809_01029_amd/csrc/kernels.hip",
                  "paper_1809_01029_amd/csrc/kernels_ext.hip", "paper_1809_01029_amd/csrc/internal.h",
                  "paper_1809_01029_amd/csrc/mech.cpp", "paper_1809_01029_amd/csrc/api.cpp",
                  "paper_1809_01029_amd/csrc/kernels_conv.hip", "paper_1809_01029_amd/csrc/kernels_ext_conv.hip"]


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, form, layout, n, shape):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload, or None if there is none, it was taken with another launch
    shape, or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pj_kernel_{workload}_{form}_{layout}_{shape[0]}x{shape[1]}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("kernel_sources_sha256") != kernel_sources_sha256() or int(kv["n_states"]) != n:
            return None
        if tuple(int(v) for v in kv["launch_shape"].split(",")) != tuple(shape):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def ragged_batch(api, synth, torch, tmp, args, stream, timeit):
    """Source terms and adjoint over 3,000 / 70,000 / 20,000 states of the 13-,
    53- and 111-species mechanisms: three per-mechanism launches (each with
    its own autotuned shape) against one ragged-batch launch and its HIP
    graph."""
    segs = []
    for name, count, seed in (("ns13", 3000, 2013), ("ns53", 70000, 2053), ("ns111", 20000, 2111)):
        w = synth.WORKLOADS[name]
        mm = synth.workload_mechanism(name)
        pth = os.path.join(tmp, f"ragged_{name}.pjm")
        synth.write_mechanism(mm, pth)
        st = synth.make_states(mm, count, seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
        x, p = synth.pack_state(st, args.form, args.layout)
        me = api.load_mechanism(pth)
        xs = torch.from_numpy(x).cuda()
        segs.append(dict(mech=me, xs=xs, ps=torch.from_numpy(p).cuda(), d=torch.empty_like(xs),
                         v=torch.randn_like(xs), jtv=torch.empty_like(xs),
                         g=torch.empty((3, me.n_reactions), dtype=torch.float64, device="cuda")))
    out = {"states": [3000, 70000, 20000]}
    for mode in ("source", "adjoint"):
        for sg in segs:
            if mode == "source":
                api.autotune(sg["mech"], sg["xs"], sg["ps"], args.form, args.layout, mode="source", reps=2,
                             stream=stream)

        def plain():
            for sg in segs:
                if mode == "source":
                    api.eval_source(sg["mech"], sg["xs"], sg["ps"], args.form, args.layout, out=sg["d"],
                                    stream=stream)
                else:
                    api.eval_adjoint(sg["mech"], sg["xs"], sg["ps"], sg["v"], args.form, args.layout,
                                     jtv=sg["jtv"], grad=sg["g"], stream=stream)
        if mode == "adjoint":
            for sg in segs:
                api.autotune(sg["mech"], sg["xs"], sg["ps"], args.form, args.layout, mode="adjoint", reps=2,
                             stream=stream)
        b = api.Batch()
        for sg in segs:
            if mode == "source":
                b.add(sg["mech"], sg["xs"], sg["ps"], args.layout, dstate=sg["d"])
            else:
                b.add(sg["mech"], sg["xs"], sg["ps"], args.layout, out=sg["jtv"], v=sg["v"], grad=sg["g"])
        # the batch autotuner chooses between one persistent launch (at its
        # best shape) and one launch per segment (at each mechanism's shape);
        # three timed launches per candidate keep the choice above the noise
        b.autotune(mode, args.form, args.layout, reps=3, stream=stream)
        chosen = b.strategy(mode)
        # medians of 7 timings of 20 back-to-back calls each (the strategies
        # differ by a few per cent; 20 calls amortise the first launch of a
        # timing onto an idle GPU, which costs a graph launch more)
        t_plain = timeit(plain, k=20, trials=7)
        t_batch = timeit(lambda: b.eval(mode, args.form, args.layout, stream=stream), k=20, trials=7)
        t_graph = timeit(lambda: b.eval(mode, args.form, args.layout, graph=True, stream=stream), k=20, trials=7)
        b.set_strategy(mode, not chosen)
        t_other = timeit(lambda: b.eval(mode, args.form, args.layout, stream=stream), k=20, trials=7)
        t_persist, t_perseg = (t_other, t_batch) if chosen else (t_batch, t_other)
        out[mode] = {"per_mechanism_ms": round(t_plain, 4), "batch_ms": round(t_batch, 4),
                     "graph_ms": round(t_graph, 4),
                     "batch_strategy": "per_segment" if chosen else "persistent",
                     "persistent_launch_ms": round(t_persist, 4), "per_segment_launches_ms": round(t_perseg, 4),
                     "persistent_shape": list(b.launch_shape(mode))}
        b.close()
    for sg in segs:
        sg["mech"].close()
    out["many_small"] = many_small_batch(api, synth, torch, tmp, args, stream, timeit)
    return out


def many_small_batch(api, synth, torch, tmp, args, stream, timeit, nseg=16, count=1024):
    """The launch-latency-bound regime: 16 segments of 1,024 states of the
    13-species mechanism (separate state draws), source terms and sparse
    Jacobian: one launch per segment against the batch (autotuned strategy)
    and its graph."""
    w = synth.WORKLOADS["ns13"]
    mm = synth.workload_mechanism("ns13")
    pth = os.path.join(tmp, "small_ns13.pjm")
    synth.write_mechanism(mm, pth)
    me = api.load_mechanism(pth)
    segs = []
    for k in range(nseg):
        st = synth.make_states(mm, count, 3000 + k, T_range=w.T_range, P_range_atm=w.P_range_atm)
        x, p = synth.pack_state(st, args.form, args.layout)
        xs = torch.from_numpy(x).cuda()
        segs.append(dict(xs=xs, ps=torch.from_numpy(p).cuda(), d=torch.empty_like(xs),
                         j=torch.empty((me.nnz, count) if args.layout == "F" else (count, me.nnz),
                                       dtype=torch.float64, device="cuda")))
    out = {"segments": nseg, "states_per_segment": count}
    for mode in ("source", "sparse"):
        api.autotune(me, segs[0]["xs"], segs[0]["ps"], args.form, args.layout, mode=mode, reps=2, stream=stream)

        def plain():
            for sg in segs:
                if mode == "source":
                    api.eval_source(me, sg["xs"], sg["ps"], args.form, args.layout, out=sg["d"], stream=stream)
                else:
                    api.eval_jacobian_sparse(me, sg["xs"], sg["ps"], args.form, args.layout, out=sg["j"],
                                             dstate=sg["d"], stream=stream)
        b = api.Batch()
        for sg in segs:
            b.add(me, sg["xs"], sg["ps"], args.layout, out=sg["j"] if mode == "sparse" else None, dstate=sg["d"])
        b.autotune(mode, args.form, args.layout, reps=3, stream=stream)
        out[mode] = {"per_segment_launches_ms": round(timeit(plain, k=20, trials=5), 4),
                     "batch_ms": round(timeit(lambda: b.eval(mode, args.form, args.layout, stream=stream), k=20,
                                              trials=5), 4),
                     "graph_ms": round(timeit(lambda: b.eval(mode, args.form, args.layout, graph=True,
                                                             stream=stream), k=20, trials=5), 4),
                     "batch_strategy": "per_segment" if b.strategy(mode) else "persistent",
                     "persistent_shape": list(b.launch_shape(mode))}
        b.close()
    me.close()
    return out


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of ``nbytes``, ``reps`` times."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def fp64_calibration(n=1 << 22, reps=16):
    """The four launches of pj_calibrate_fp64 (exp, log, log10, loop alone)
    whose FP64 counters give the device's weight of each function."""
    import torch
    from paper_1809_01029_amd import api
    x = torch.linspace(0.5, 1.5, n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    res = {}
    for fn in ("exp", "log", "log10", "none"):
        api.calibrate_fp64(fn, x, reps, out=y)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        api.calibrate_fp64(fn, x, reps, out=y)
        b.record()
        torch.cuda.synchronize()
        res[fn] = round(a.elapsed_time(b), 4)
    print(json.dumps({"calibration_calls": n * reps, "ms": res}), flush=True)


def fp64_weights():
    """FP64 operations of one call of the device's exp, log and log10, from
    the committed counter summary of the calibration launches, or None."""
    path = os.path.join(ROOT, "profiles", "fp64_transcendental_weights.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        return {f: float(kv[f"w_{f}"]) for f in ("exp", "log", "log10")}
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ns111")
    ap.add_argument("--n-states", type=int, default=0, help="override the workload's state count")
    ap.add_argument("--form", default="conp", choices=["conp", "conv"])
    ap.add_argument("--layout", default="C", choices=["F", "C"])
    ap.add_argument("--cpu-sample", type=int, default=12288, help="states timed on the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape instead of autotuning it first")
    ap.add_argument("--launch", default="",
                    help="S,W: fix the launch shape (states and waves per workgroup) instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (traffic-counter reference)")
    ap.add_argument("--fp64-calibration", action="store_true",
                    help="run only the FP64 weight calibration launches of exp, log and log10")
    ap.add_argument("--source-only", action="store_true",
                    help="time the source-term kernel alone (for its profiles), not the benchmark step")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time the adjoint kernel alone (J^T v and parameter sums, for its profiles)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); states are independent, "
              "so more GPUs would each run this same benchmark on their own share.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.fp64_calibration:
        fp64_calibration()
        return

    import numpy as np
    import torch

    from paper_1809_01029_amd import api, synth

    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    n = args.n_states or w.n_states
    tmp = tempfile.mkdtemp(prefix="pjbench_")
    path = os.path.join(tmp, f"{args.workload}.pjm")
    t0 = time.time()
    m = synth.workload_mechanism(args.workload)
    synth.write_mechanism(m, path)
    st = synth.make_states(m, n, w.state_seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
    x, p = synth.pack_state(st, args.form, args.layout)
    log(f"inputs: {args.workload} Ns={m.n_species} Nr={m.n_reactions} n={n} ({time.time() - t0:.1f}s)")

    mech = api.load_mechanism(path)
    N, nnz = mech.N, mech.nnz
    xs = torch.from_numpy(x).cuda()
    ps = torch.from_numpy(p).cuda()
    dstate = torch.empty_like(xs)
    jshape = (nnz, n) if args.layout == "F" else (n, nnz)
    jac = torch.empty(jshape, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    tuned = None
    if args.launch:
        S_, W_ = (int(v) for v in args.launch.split(","))
        mech.set_launch(S_, W_)
        args.no_autotune = True
    if args.source_only:
        # the source-term kernel alone, in the shape its autotuner picks
        if not args.no_autotune:
            api.autotune(mech, xs, ps, args.form, args.layout, mode="source", reps=2, stream=stream)
        for _ in range(args.warmup):
            api.eval_source(mech, xs, ps, args.form, args.layout, out=dstate, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            api.eval_source(mech, xs, ps, args.form, args.layout, out=dstate, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"source_only_ms": round(t, 4), "states_per_s": n / (t * 1e-3), "n_states": n,
                          "workload": args.workload, "launch_shape": list(mech.launch_shape(0))}), flush=True)
        return
    if args.adjoint_only:
        # the adjoint kernel alone (v ~ N(0, 1), seed 7), in the shape its
        # autotuner picks unless --launch gives one
        g = torch.Generator(device="cpu").manual_seed(7)
        vs = torch.randn(xs.shape, generator=g, dtype=torch.float64).cuda()
        jtv = torch.empty_like(xs)
        grad = torch.empty((3, mech.n_reactions), dtype=torch.float64, device="cuda")
        if not args.no_autotune:
            api.autotune(mech, xs, ps, args.form, args.layout, mode="adjoint", reps=2, stream=stream)
        for _ in range(args.warmup):
            api.eval_adjoint(mech, xs, ps, vs, args.form, args.layout, jtv=jtv, grad=grad, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            api.eval_adjoint(mech, xs, ps, vs, args.form, args.layout, jtv=jtv, grad=grad, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"adjoint_ms": round(t, 4), "states_per_s": n / (t * 1e-3), "n_states": n,
                          "workload": args.workload, "launch_shape": list(mech.launch_shape(3))}), flush=True)
        return
    if not args.no_autotune:
        # outside the timed region: pick the fastest launch shape for this batch
        t0 = time.time()
        tuned = api.autotune(mech, xs, ps, args.form, args.layout, mode="sparse", reps=2, stream=stream)
        log(f"autotuned launch shape {tuned[:2]} ({tuned[2]:.3f} ms) in {time.time() - t0:.1f}s")

    def step():
        api.eval_jacobian_sparse(mech, xs, ps, args.form, args.layout, out=jac, dstate=dstate,
                                 stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms = ms_total / args.steps
    value = n / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.4f} ms/step, {value:.4e} states/s")

    # algorithmic HBM bytes per state: state + parameter in, source terms and
    # CSR values out (mechanism tables and intermediates excluded)
    bytes_state = 8 * (N + 1) + 8 * N + 8 * nnz
    achieved = bytes_state * n / (ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.form, args.layout, n, mech.launch_shape(1))
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_state": bytes_state, "algorithmic_bytes_per_launch": bytes_state * n}

    variants = {}
    if not args.no_variants:
        def timeit(fn, k=5, trials=1):
            """ms per call of k back-to-back calls after one untimed call;
            the median over ``trials`` such timings"""
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(trials):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(k):
                    fn()
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b) / k)
            return sorted(ts)[len(ts) // 2]
        out_src = torch.empty_like(xs)
        if not args.no_autotune:
            api.autotune(mech, xs, ps, args.form, args.layout, mode="source", reps=2, stream=stream)
        t = timeit(lambda: api.eval_source(mech, xs, ps, args.form, args.layout, out=out_src, stream=stream))
        variants["source_only"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3),
                                   "launch_shape": list(mech.launch_shape(0))}
        del out_src
        if N * N * n * 8 < 60e9:
            dshape = (N, N, n) if args.layout == "F" else (n, N, N)
            dj = torch.empty(dshape, dtype=torch.float64, device="cuda")
            if not args.no_autotune:
                api.autotune(mech, xs, ps, args.form, args.layout, mode="dense", reps=1, stream=stream)
            t = timeit(lambda: api.eval_jacobian_dense(mech, xs, ps, args.form, args.layout, out=dj,
                                                       dstate=dstate, stream=stream), k=3)
            db = (8 * (2 * N + 1) + 8 * N * N) * n
            variants["dense_jacobian"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3), "layout": args.layout,
                                          "hbm_GBps": db / (t * 1e-3) / 1e9,
                                          "frac": round(db / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del dj
            # the other state layout (F: [s + n (i + N j)]; C: [s][i][j])
            ol = "C" if args.layout == "F" else "F"
            xo, po = synth.pack_state(st, args.form, ol)
            xso, pso = torch.from_numpy(xo).cuda(), torch.from_numpy(po).cuda()
            del xo
            dj = torch.empty((N, N, n) if ol == "F" else (n, N, N), dtype=torch.float64, device="cuda")
            do = torch.empty_like(xso)
            if not args.no_autotune:
                api.autotune(mech, xso, pso, args.form, ol, mode="dense", reps=1, stream=stream)
            t = timeit(lambda: api.eval_jacobian_dense(mech, xso, pso, args.form, ol, out=dj, dstate=do,
                                                       stream=stream), k=3)
            variants[f"dense_jacobian_layout_{ol}"] = {
                "ms": round(t, 4), "states_per_s": n / (t * 1e-3), "hbm_GBps": db / (t * 1e-3) / 1e9,
                "frac": round(db / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "launch_shape": list(mech.launch_shape(2))}
            del dj, xso, pso, do
            if not args.no_autotune:
                api.autotune(mech, xs, ps, args.form, args.layout, mode="dense", reps=1, stream=stream)
        other = "conv" if args.form == "conp" else "conp"
        x2, p2 = synth.pack_state(st, other, args.layout)
        xs2, ps2 = torch.from_numpy(x2).cuda(), torch.from_numpy(p2).cuda()
        t = timeit(lambda: api.eval_jacobian_sparse(mech, xs2, ps2, other, args.layout, out=jac,
                                                    dstate=dstate, stream=stream))
        variants[f"{other}_sparse"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3)}
        if N * N * n * 8 < 60e9:
            # the dense Jacobian in the other form as well (same layout)
            dj = torch.empty((N, N, n) if args.layout == "F" else (n, N, N), dtype=torch.float64, device="cuda")
            t = timeit(lambda: api.eval_jacobian_dense(mech, xs2, ps2, other, args.layout, out=dj,
                                                       dstate=dstate, stream=stream), k=3)
            db = (8 * (2 * N + 1) + 8 * N * N) * n
            variants[f"dense_jacobian_{other}"] = {
                "ms": round(t, 4), "states_per_s": n / (t * 1e-3), "layout": args.layout,
                "hbm_GBps": db / (t * 1e-3) / 1e9, "frac": round(db / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "launch_shape": list(mech.launch_shape(2))}
            del dj
        del xs2, ps2
        ol = "C" if args.layout == "F" else "F"
        x3, p3 = synth.pack_state(st, args.form, ol)
        xs3, ps3 = torch.from_numpy(x3).cuda(), torch.from_numpy(p3).cuda()
        jac3 = torch.empty((nnz, n) if ol == "F" else (n, nnz), dtype=torch.float64, device="cuda")
        d3 = torch.empty_like(xs3)
        t = timeit(lambda: api.eval_jacobian_sparse(mech, xs3, ps3, args.form, ol, out=jac3, dstate=d3,
                                                    stream=stream))
        variants[f"layout_{ol}_sparse"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3)}
        del xs3, ps3, jac3, d3
        # fixed-order accumulation (bitwise reproducible at any one launch
        # shape), at the shape its own autotuning picks (outside the timing)
        mdet = api.load_mechanism(path, options=api.OPT_DETERMINISTIC)
        api.autotune(mdet, xs, ps, args.form, args.layout, mode="sparse", reps=1, stream=stream)
        t = timeit(lambda: api.eval_jacobian_sparse(mdet, xs, ps, args.form, args.layout, out=jac,
                                                    dstate=dstate, stream=stream))
        variants["deterministic_sparse"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3),
                                            "cost_vs_default": round(t / ms, 3),
                                            "launch_shape": list(mdet.launch_shape(1))}
        del mdet
        if args.workload == "ns111" and not args.n_states:
            # the 53-species configuration at its full size (1,048,576 states)
            w53 = synth.WORKLOADS["ns53"]
            m53 = synth.workload_mechanism("ns53")
            p53 = os.path.join(tmp, "ns53.pjm")
            synth.write_mechanism(m53, p53)
            st53 = synth.make_states(m53, w53.n_states, w53.state_seed, T_range=w53.T_range,
                                     P_range_atm=w53.P_range_atm)
            x4, p4 = synth.pack_state(st53, args.form, args.layout)
            del st53
            mech53 = api.load_mechanism(p53)
            xs4, ps4 = torch.from_numpy(x4).cuda(), torch.from_numpy(p4).cuda()
            del x4
            n4 = w53.n_states
            jac4 = torch.empty((mech53.nnz, n4) if args.layout == "F" else (n4, mech53.nnz), dtype=torch.float64,
                               device="cuda")
            d4 = torch.empty_like(xs4)
            if not args.no_autotune:
                api.autotune(mech53, xs4, ps4, args.form, args.layout, mode="sparse", reps=1, stream=stream)
            t = timeit(lambda: api.eval_jacobian_sparse(mech53, xs4, ps4, args.form, args.layout, out=jac4,
                                                        dstate=d4, stream=stream), k=3)
            b4 = 8 * (mech53.N + 1) + 8 * mech53.N + 8 * mech53.nnz
            variants["ns53_1M_sparse"] = {"ms": round(t, 4), "states_per_s": n4 / (t * 1e-3),
                                          "hbm_frac": b4 * n4 / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                          "launch_shape": list(mech53.launch_shape(1))}
            del xs4, ps4, jac4, d4
            mech53.close()
            # the 360-species configuration at its full size (16,384 states,
            # T 700..1800 K, P 10..60 atm): source terms + sparse Jacobian
            w360 = synth.WORKLOADS["ns360"]
            m360 = synth.workload_mechanism("ns360")
            p360 = os.path.join(tmp, "ns360.pjm")
            synth.write_mechanism(m360, p360)
            st360 = synth.make_states(m360, w360.n_states, w360.state_seed, T_range=w360.T_range,
                                      P_range_atm=w360.P_range_atm)
            x7, p7 = synth.pack_state(st360, args.form, args.layout)
            del st360
            mech360 = api.load_mechanism(p360)
            xs7, ps7 = torch.from_numpy(x7).cuda(), torch.from_numpy(p7).cuda()
            n7 = w360.n_states
            jac7 = torch.empty((mech360.nnz, n7) if args.layout == "F" else (n7, mech360.nnz), dtype=torch.float64,
                               device="cuda")
            d7 = torch.empty_like(xs7)
            if not args.no_autotune:
                api.autotune(mech360, xs7, ps7, args.form, args.layout, mode="sparse", reps=1, stream=stream)
            t = timeit(lambda: api.eval_jacobian_sparse(mech360, xs7, ps7, args.form, args.layout, out=jac7,
                                                        dstate=d7, stream=stream), k=5)
            if not args.no_autotune:
                api.autotune(mech360, xs7, ps7, args.form, args.layout, mode="source", reps=1, stream=stream)
            ts = timeit(lambda: api.eval_source(mech360, xs7, ps7, args.form, args.layout, out=d7, stream=stream))
            b7 = 8 * (mech360.N + 1) + 8 * mech360.N + 8 * mech360.nnz
            variants["ns360_16k_sparse"] = {"ms": round(t, 4), "states_per_s": n7 / (t * 1e-3), "nnz": mech360.nnz,
                                            "bytes_per_state": b7,
                                            "hbm_frac": round(b7 * n7 / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                            "launch_shape": list(mech360.launch_shape(1)),
                                            "source_only_ms": round(ts, 4),
                                            "source_launch_shape": list(mech360.launch_shape(0))}
            del xs7, ps7, jac7, d7
            mech360.close()
        # adjoint (J^T v + Arrhenius-parameter sums) on the same batch
        if not args.no_autotune:
            api.autotune(mech, xs, ps, args.form, args.layout, mode="adjoint", reps=1, stream=stream)
        vv = torch.randn_like(xs)
        jtv = torch.empty_like(xs)
        grad = torch.empty((3, m.n_reactions), dtype=torch.float64, device="cuda")
        t = timeit(lambda: api.eval_adjoint(mech, xs, ps, vv, args.form, args.layout, jtv=jtv, grad=grad,
                                            stream=stream))
        variants["adjoint"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3),
                               "launch_shape": list(mech.launch_shape(3)),
                               "vs_sparse_jacobian": round(t / ms, 3)}
        del vv, jtv, grad
        # the Jacobian variants of the paper on the same batch: approximate
        # form, column-ordered values, run-time slot search (the lookup the
        # static map replaces)
        for label, opt in (("approximate_jacobian", api.OPT_APPROX_JACOBIAN), ("ccs_output", api.OPT_CCS),
                           ("run_time_slot_search", api.OPT_LINEAR_SEARCH)):
            mv = api.load_mechanism(path, options=opt)
            mv.set_launch(*mech.launch_shape(1))
            jv = torch.empty((mv.nnz, n) if args.layout == "F" else (n, mv.nnz), dtype=torch.float64,
                             device="cuda")
            t = timeit(lambda: api.eval_jacobian_sparse(mv, xs, ps, args.form, args.layout, out=jv, dstate=dstate,
                                                        stream=stream), k=3)
            variants[label] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3), "nnz": mv.nnz,
                               "vs_static_csr": round(t / ms, 3)}
            del jv
            mv.close()
        if args.workload == "ns111" and not args.n_states:
            # the 13-species configuration at its size (1,024 states): launch
            # latency bound, reported per call
            w13 = synth.WORKLOADS["ns13"]
            m13 = synth.workload_mechanism("ns13")
            p13 = os.path.join(tmp, "ns13.pjm")
            synth.write_mechanism(m13, p13)
            st13 = synth.make_states(m13, w13.n_states, w13.state_seed, T_range=w13.T_range,
                                     P_range_atm=w13.P_range_atm)
            x6, p6 = synth.pack_state(st13, args.form, args.layout)
            mech13 = api.load_mechanism(p13)
            xs6, ps6 = torch.from_numpy(x6).cuda(), torch.from_numpy(p6).cuda()
            j6 = torch.empty((mech13.nnz, w13.n_states) if args.layout == "F" else (w13.n_states, mech13.nnz),
                             dtype=torch.float64, device="cuda")
            d6 = torch.empty_like(xs6)
            if not args.no_autotune:
                api.autotune(mech13, xs6, ps6, args.form, args.layout, mode="sparse", reps=3, stream=stream)
            t = timeit(lambda: api.eval_jacobian_sparse(mech13, xs6, ps6, args.form, args.layout, out=j6, dstate=d6,
                                                        stream=stream), k=50)
            variants["ns13_1024_sparse"] = {"us_per_call": round(t * 1e3, 2),
                                            "states_per_s": w13.n_states / (t * 1e-3),
                                            "launch_shape": list(mech13.launch_shape(1))}
            del xs6, ps6, j6, d6
            mech13.close()
        # saturation: states/s of the same launch against the batch size (the
        # first k states of this batch)
        sat = {}
        for k in (100, 1000, 10000, 30000, 100000, n):
            if k > n:
                continue
            xk = xs[:k] if args.layout == "C" else xs[:, :k].contiguous()
            pk = ps[:k]
            jk = torch.empty((nnz, k) if args.layout == "F" else (k, nnz), dtype=torch.float64, device="cuda")
            dk = torch.empty_like(xk)
            t = timeit(lambda: api.eval_jacobian_sparse(mech, xk, pk, args.form, args.layout, out=jk, dstate=dk,
                                                        stream=stream), k=10 if k < n else 3)
            sat[str(k)] = {"ms": round(t, 4), "states_per_s": k / (t * 1e-3)}
            del xk, jk, dk
        variants["saturation_sparse"] = sat
        # with the inputs copied in from pinned host memory and the outputs
        # (source terms and CSR values) copied back, per step (not `value`);
        # a host that cannot pin that much memory records the error instead
        try:
            hx = torch.empty(xs.shape, dtype=torch.float64, pin_memory=True)
            hp = torch.empty(ps.shape, dtype=torch.float64, pin_memory=True)
            hj = torch.empty(jac.shape, dtype=torch.float64, pin_memory=True)
            hd = torch.empty(dstate.shape, dtype=torch.float64, pin_memory=True)
            hx.copy_(xs)
            hp.copy_(ps)

            def pcie_step():
                xs.copy_(hx, non_blocking=True)
                ps.copy_(hp, non_blocking=True)
                api.eval_jacobian_sparse(mech, xs, ps, args.form, args.layout, out=jac, dstate=dstate, stream=stream)
                hj.copy_(jac, non_blocking=True)
                hd.copy_(dstate, non_blocking=True)
            t = timeit(pcie_step, k=2)
            variants["pcie_inclusive_sparse"] = {"ms": round(t, 4), "states_per_s": n / (t * 1e-3),
                                                 "bytes_over_pcie": int((xs.numel() + ps.numel() + jac.numel()
                                                                         + dstate.numel()) * 8)}
            del hx, hp, hj, hd
        except (RuntimeError, MemoryError) as exc:
            variants["pcie_inclusive_sparse"] = {"error": str(exc)[:200]}
        if args.workload == "ns111" and not args.n_states:
            variants["ragged_13_53_111"] = ragged_batch(api, synth, torch, tmp, args, stream, timeit)
            # the same size with every reaction type (SRI, chemically activated,
            # P-Log, Chebyshev besides the default mix), on its own states
            wx = synth.WORKLOADS["ns111x"]
            mx = synth.workload_mechanism("ns111x")
            px = os.path.join(tmp, "ns111x.pjm")
            synth.write_mechanism(mx, px)
            stx = synth.make_states(mx, wx.n_states, wx.state_seed, T_range=wx.T_range, P_range_atm=wx.P_range_atm)
            x5, p5 = synth.pack_state(stx, args.form, args.layout)
            del stx
            mechx = api.load_mechanism(px)
            xs5, ps5 = torch.from_numpy(x5).cuda(), torch.from_numpy(p5).cuda()
            jac5 = torch.empty((mechx.nnz, wx.n_states) if args.layout == "F" else (wx.n_states, mechx.nnz),
                               dtype=torch.float64, device="cuda")
            d5 = torch.empty_like(xs5)
            if not args.no_autotune:
                api.autotune(mechx, xs5, ps5, args.form, args.layout, mode="sparse", reps=1, stream=stream)
            t = timeit(lambda: api.eval_jacobian_sparse(mechx, xs5, ps5, args.form, args.layout, out=jac5,
                                                        dstate=d5, stream=stream), k=3)
            ts = timeit(lambda: api.eval_source(mechx, xs5, ps5, args.form, args.layout, out=d5, stream=stream))
            variants["all_reaction_types_ns111x"] = {
                "ms": round(t, 4), "states_per_s": wx.n_states / (t * 1e-3), "nnz": mechx.nnz,
                "launch_shape": list(mechx.launch_shape(1)), "source_only_ms": round(ts, 4),
                "vs_ns111": round(t / ms, 3)}
            del xs5, ps5, jac5, d5
            mechx.close()
        log(f"variants: {json.dumps(variants)}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        k = min(args.cpu_sample, n)
        xc, pc = synth.pack_state(st, args.form, "C")
        xc, pc = np.ascontiguousarray(xc[:k]), pc[:k]
        o = oracle.Oracle(path)

        def run_oracle(ix):
            o.source(xc[ix], pc[ix], args.form)
            o.jacobian(xc[ix], pc[ix], args.form)
        # one host core on a tenth of the sample, then every core of the
        # host's share on the whole sample, 10 times (the paper's mean of 10
        # runs; the oracle's C calls release the interpreter lock, so threads
        # run in parallel)
        k1 = max(1, k // 10)
        t0 = time.perf_counter()
        run_oracle(np.arange(k1))
        dt1 = (time.perf_counter() - t0) * k / k1
        threads = max(1, min(16, os.cpu_count() or 1))
        runs = []
        with concurrent.futures.ThreadPoolExecutor(threads) as ex:
            for _ in range(10):
                t0 = time.perf_counter()
                list(ex.map(run_oracle, np.array_split(np.arange(k), threads)))
                runs.append(time.perf_counter() - t0)
        dt = float(np.mean(runs))
        host = platform.processor() or platform.machine()
        try:
            with open("/proc/cpuinfo") as fh:
                host = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), host)
        except OSError:
            pass
        cpu = {"value": k / dt, "unit": "states/s", "cores": threads, "kind": "oracle",
               "serial_value": k / dt1, "host_cpu": host, "host_cpus_visible": os.cpu_count(),
               "runs": 10, "run_s": [round(r, 3) for r in runs],
               "sample": f"first {k} of the {n} {args.workload} states: source terms + analytical "
                         f"Jacobian (dense, holding the CSR values), FP64 oracle on {threads} host threads, "
                         f"mean of 10 runs {dt:.2f} s; one thread on the first {k1} states, scaled to {k} "
                         f"({dt1:.1f} s, serial_value)"}
        # operation count of the source terms (the oracle's definitions without
        # the derivatives, ln T once) for the FP64 roofline of the source-only
        # kernel, weighted by the device's own exp / log / log10
        ops = [o.source_ops(xc[i], pc[i], args.form) for i in range(min(8, k))]
        wts = fp64_weights()
        if "source_only" in variants:
            so = variants["source_only"]
            if wts is None:
                so["roofline"] = None
            else:
                fl = float(np.mean([q["flops"] + wts["exp"] * q["exp"] + wts["log"] * q["log"]
                                    + wts["log10"] * q["log10"] for q in ops]))
                ach = fl * n / (so["ms"] * 1e-3) / 1e12
                so["roofline"] = {"bound": "fp64", "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                                  "flops_per_state": round(fl, 1), "ops_per_state": ops[0],
                                  "weights": wts}
        log(f"cpu oracle: {cpu['value']:.2f} states/s on {threads} threads, {k / dt1:.2f} on one, {k} states")

    out = {
        "metric": METRIC, "value": value, "unit": "states/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: synthetic {m.n_species} species / {m.n_reactions} "
                               f"reactions, {n} states, {args.form.upper()}, layout {args.layout}, "
                               f"fused source terms + sparse CSR Jacobian",
                   "n_species": m.n_species, "n_reactions": m.n_reactions, "n_states": n, "nnz": nnz,
                   "form": args.form, "layout": args.layout,
                   "launch_shape": {"states_per_workgroup": mech.launch_shape(1)[0],
                                    "waves_per_workgroup": mech.launch_shape(1)[1],
                                    "autotuned": tuned is not None}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
