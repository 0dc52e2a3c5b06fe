"""Compile libhydro.so (HIP, gfx950) in-tree with hipcc: every source to an
object in parallel, then one link."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhydro.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["capi.hip", "mhm_fwd.hip", "mhm_fwd_g2.hip", "mhm_fwd_ext.hip", "mhm_batched.hip", "mhm_adj.hip", "aux_kernels.hip", "scheme_ext.hip",
           "fallback.hip", "amr.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # one rounding per source expression, identical at every inlined site
    "-ffp-contract=on",
    # keep the compiler from forming packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build_library(extra_flags=(), verbose=False, jobs=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    tag = "%d" % os.getpid()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(OBJ, src.replace(".hip", ".%s.o" % tag))
        cmd = [hipcc, *HIPCC_FLAGS, *extra_flags, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        return obj

    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp" + tag
    try:
        subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    build_library(sys.argv[1:], verbose=True)
