"""Builds libchemstep.so (all HIP sources under csrc/) for gfx950 with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libchemstep.so")
OBJ = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# per-source extra flags: the network kernels keep MFMA accumulators in the
# architectural VGPRs (measured faster than the AGPR form for these tiles)
EXTRA = {"ann_kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
         "profile.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(src, jobs_out):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
    return obj, subprocess.Popen(cmd)


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    procs = []
    for src in sources():
        obj, pr = _compile(src, None)
        procs.append((src, obj, pr))
    objs = []
    for src, obj, pr in procs:
        if pr.wait() != 0:
            raise RuntimeError("hipcc failed on " + src)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
