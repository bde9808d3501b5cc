"""Build libsawave.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2511_18071_amd.build

Every HIP source is compiled for gfx950 only; packed FP32 instructions are disabled for the
device code. The library lands next to this file, where the Python binding loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsawave.so")
SOURCES = ["solve64.hip", "solve32.hip", "api.hip", "server.hip", "static_apply.hip", "operator3d.hip", "closedloop.hip", "setup.cpp", "ilu.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(ROOT, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    cmds = []
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc(), *common, f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                   "-packed-fp32-ops", "-x", "hip", "-c", path, "-o", obj]
        else:
            cmd = [hipcc(), *common, "-x", "c++", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the kernel translation units are large: compile them side by side
    procs = [subprocess.Popen(c) for c in cmds]
    codes = [p.wait() for p in procs]
    if any(codes):
        raise subprocess.CalledProcessError(next(c for c in codes if c), "hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
