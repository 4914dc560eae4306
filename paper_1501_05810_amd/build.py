"""Build ``libnbgs.so`` (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled with ``-ffp-contract=off`` so that FP64
expressions are evaluated exactly as written (the contact set and the FP64
sweeps are compared bit for bit with a plain sequential definition), and with
packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnbgs.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("NBGS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.hip", "sort.hip", "detect.hip", "colour.hip", "sweep.hip", "mlp.hip", "warmstart.hip", "tune.hip",
           "batch.hip", "subdomain.hip", "composite.hip"]

COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link the shared library."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for src in sources():
        obj = os.path.join(BUILD_DIR, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([cc, *COMMON, "-c", src, "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
        return r.stderr

    with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
        for msg in ex.map(run, cmds):
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [cc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    run(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
