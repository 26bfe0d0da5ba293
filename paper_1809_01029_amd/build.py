"""Build the HIP library (libpjac.so, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpjac.so")
BUILD = os.path.join(HERE, "_build")

ARCH = os.environ.get("PJ_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC, "-Wall"]
# packed FP32 instructions stay disabled in every device compile
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        sys.stderr.write(out + "\n")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in ("mech.cpp", "api.cpp", "batch.cpp", "kernels.hip", "kernels_conv.hip", "kernels_ext.hip",
                "kernels_ext_conv.hip", "calibrate.hip", "noalloc.hip"):
        o = os.path.join(BUILD, src + ".o")
        # host-only translation units: no device pass
        dev = DEVICE if src.endswith(".hip") else ["--offload-host-only"]
        jobs.append(([HIPCC] + COMMON + dev + ["-c", os.path.join(CSRC, src), "-o", o], o))
    # the translation units compile in parallel (the two kernel sets dominate)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, cmd) for cmd, _ in jobs]:
            f.result()
    objs = [o for _, o in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC] + DEVICE + ["-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
