"""Build libhbi.so (HIP for gfx950) in the package directory.

    python -m paper_2210_02698_amd.build        # or build() from Python

The library is compiled with hipcc for gfx950 only.  Packed FP32 vector
instructions are disabled (-packed-fp32-ops) for every HIP translation unit.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhbi.so")

HIP_SOURCES = ["hbi_kernels.hip", "hbi_apply.hip", "hbi_multi.hip", "hbi_inclusion.hip",
               "hbi_s2v.hip", "hbi_tabulate.hip", "hbi_lib.hip"]
CPP_SOURCES = ["hbi_geometry.cpp"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    hipflags = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops", "-munsafe-fp-atomics"]
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append([hipcc, *common, *hipflags, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append(["g++", *common, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    failed = []
    for cmd, p in zip(cmds, procs):
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            failed.append((cmd, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(" ".join(c) + "\n" + o for c, o in failed)
        raise RuntimeError("libhbi build failed:\n" + msg)
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
