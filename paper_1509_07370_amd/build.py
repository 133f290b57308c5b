"""Build the HIP library libbh.so for gfx950 in-tree with hipcc.

Run as ``python -m paper_1509_07370_amd.build``.  Compiles every source under
csrc/ into paper_1509_07370_amd/libbh.so.  Packed fp32 instructions are
disabled on purpose (-packed-fp32-ops): the compiler would otherwise form
v_pk_* fp32 operations from scalar float code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbh.so")
SOURCES = ["bh_api.cpp", "bh_topology.cpp", "bh_mlp_api.cpp", "bh_batch_api.cpp", "bh_kernels.hip", "bh_mlp.hip",
           "bh_periodic.hip", "bh_ewald_series.cpp",
           "bh_static.hip"]
ARCH = os.environ.get("BH_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "-Wall", "--offload-arch=" + ARCH, "-I" + os.path.join(ROOT, "include"),
            "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        cmd = [cc, *flags(), "-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [cc, *flags(), "-x", "hip", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
