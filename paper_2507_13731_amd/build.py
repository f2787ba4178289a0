"""Build the HIP library libqlra.so for gfx950 in-tree with hipcc.

Every HIP source is compiled for gfx950 only.  Packed-FP32 instruction selection is disabled
(-packed-fp32-ops); the sketch generator is compiled without FP contraction so that its
operation sequence is exactly the written one.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqlra.so")

SOURCES = ["omega.hip", "qgemm.hip", "lowp.hip", "chol.hip", "qsvd.hip", "heig.hip", "heig_big.hip", "util.hip",
           "complete.hip", "qlra.cpp", "noalloc.hip"]
COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
PER_FILE = {"omega.hip": ["-ffp-contract=off"]}


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    cmd = ["hipcc", "-c"] + COMMON + PER_FILE.get(src, []) + [os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(msgs)))
    return obj, "\n".join(msgs)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    for obj, msg in results:
        if verbose and msg.strip():
            print(msg)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "--offload-arch=gfx950", "-o", tmp] + [o for o, _ in results]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
