"""Compiled-code check on the host (no GPU): no workgroup barrier of the
kernels may be reached while an LDS store or atomic of the same wave is still
in flight.

The reaction loop of the fixed-order mode lets the waves add to the LDS sums
in turn, one barrier per turn; the compiler did not keep the barrier's own
wait for the LDS counter on that loop's back edge, so a turn's additions
could be overtaken by the next wave's.  The kernel now waits explicitly.  This
test compiles a few instantiations for gfx950 to assembly and runs a
data-flow pass over their control-flow graph: at every s_barrier, no path
from an LDS store or atomic may avoid an `s_waitcnt lgkmcnt(0)`.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_01029_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

LDS_STORE = re.compile(r"ds_(write|add|store|max|min|or|and|xor|inc|dec|sub|swap|cmpst|pk_add)")


def pending_lds_barriers(asm: str):
    """Lines of the barriers that some path reaches with an LDS store or
    atomic not yet waited for.  Blocks start at labels; successors are the
    branch targets plus the fall-through (absent after s_branch and
    s_endpgm); the pending flag is propagated to a fixed point."""
    lines = asm.splitlines()
    blocks = [{"name": "entry", "ins": []}]
    for i, raw in enumerate(lines):
        t = raw.strip()
        m = re.match(r"^(\.LBB\d+_\d+):", t)
        if m:
            blocks.append({"name": m.group(1), "ins": []})
            continue
        if re.match(r"^; %bb\.\d+:", t):
            blocks.append({"name": t, "ins": []})
            continue
        if t and not t.startswith(";") and not t.startswith("."):
            blocks[-1]["ins"].append((i + 1, t))
    index = {b["name"]: k for k, b in enumerate(blocks)}

    def step(p, t):
        if t.startswith("s_waitcnt") and "lgkmcnt(0)" in t:
            return False
        return True if LDS_STORE.match(t) else p

    # a branch passes on the state at the branch; the fall-through the state
    # at the end of the block
    pend = [False] * len(blocks)
    changed = True
    while changed:
        changed = False
        for k, b in enumerate(blocks):
            p = pend[k]
            out = []
            for _, t in b["ins"]:
                p = step(p, t)
                m = re.match(r"s_(cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", t)
                if m:
                    out.append((index[m.group(2)], p))
            last = b["ins"][-1][1] if b["ins"] else ""
            if not (last.startswith("s_branch") or last.startswith("s_endpgm")) and k + 1 < len(blocks):
                out.append((k + 1, p))
            for j, pj in out:
                if pj and not pend[j]:
                    pend[j] = changed = True
    bad, nbar = [], 0
    for k, b in enumerate(blocks):
        p = pend[k]
        for ln, t in b["ins"]:
            if t.startswith("s_barrier"):
                nbar += 1
                if p:
                    bad.append(ln)
            p = step(p, t)
    return bad, nbar


def test_checker_flags_a_loop_back_edge_without_wait():
    # a loop whose header barrier follows, on the back edge, an LDS atomic
    # with no wait: the pattern the fixed-order kernels had
    asm = "\n".join([
        "\ts_waitcnt lgkmcnt(0)",
        "\ts_barrier",
        ".LBB0_1:",
        "\ts_barrier",
        "\tds_add_f64 v1, v[2:3]",
        "\ts_cbranch_scc1 .LBB0_1",
        "\ts_waitcnt lgkmcnt(0)",
        "\ts_barrier",
        "\ts_endpgm",
    ])
    bad, nbar = pending_lds_barriers(asm)
    assert nbar == 3 and bad == [4]
    fixed = asm.replace(".LBB0_1:\n\ts_barrier", ".LBB0_1:\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier")
    assert pending_lds_barriers(fixed)[0] == []


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_no_barrier_with_pending_lds_store(tmp_path):
    sig = ("(const DevMech, const long, const double* __restrict__, const double* __restrict__, "
           "double* __restrict__, double* __restrict__, const double* __restrict__, "
           "double* __restrict__, const int);")
    inst = [("MODE_SRC_DET", 2), ("MODE_SPARSE_DET", 2), ("MODE_SPARSE", 2), ("MODE_DENSE_U16", 2), ("MODE_ADJ", 4)]
    # the ragged batch kernel with the states per group known at run time (0)
    # and at compile time (4)
    batch = [("MODE_SPARSE", 0), ("MODE_ADJ", 4)]
    src = '#include "kernel_body.h"\nnamespace pj {\n' + "".join(
        f"template __global__ void pj_kernel<PJ_CONP, PJ_LAYOUT_C, {m}, {s}, false>{sig}\n" for m, s in inst) + "".join(
        f"template __global__ void pj_batch_kernel<PJ_CONP, PJ_LAYOUT_C, {m}, false, {su}>"
        "(const BatchSeg* __restrict__, const int, const long);\n" for m, su in batch) + "}\n"
    f = tmp_path / "isa_check.hip"
    f.write_text(src)
    out = tmp_path / "isa_check.s"
    subprocess.run([HIPCC, "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "--offload-device-only", "-S", str(f), "-o", str(out)],
                   check=True, capture_output=True, timeout=600)
    asm = out.read_text()
    bad, nbar = pending_lds_barriers(asm)
    assert nbar > 10, "expected the kernels' barriers in the assembly"
    assert bad == [], f"barriers reached with LDS stores in flight at assembly lines {bad}"
