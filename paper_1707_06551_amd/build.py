"""Build the HIP library libbie.so in-tree for gfx950 (hipcc, no JIT).

Usage: python -m paper_1707_06551_amd.build   (or __graft_entry__.build()).
Each source is compiled to an object under _build/ in parallel, then linked.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbie.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["setup.cpp", "calibrate.cpp", "api.cpp", "vsh.hip", "near.hip", "p2p.hip", "solver.hip", "coarse.hip", "mlp.hip", "rigid.hip", "field.hip", "near_rot.hip", "laplace.hip", "traction.hip", "noalloc.hip"]

# Packed FP32 instructions are disabled for all device code on purpose.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wno-unused-result",
]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip",
           "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    return obj, errs


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for (_o, e) in results:
            if e.strip():
                print(e, file=sys.stderr)
    objs = [o for (o, _e) in results]
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
