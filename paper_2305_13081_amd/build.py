"""Build step: compile the HIP sources into the in-tree shared library.

    python -m paper_2305_13081_amd.build

compiles every translation unit under ``csrc/`` (``fgcg.hip``: the C ABI and
the 2D solvers; ``fgcg3d.hip``: the 3D solvers; ``homog.hip``: the diffusion
homogenisation and concentration reconstruction; ``noalloc.hip``: the
phase-field solve without allocation) for gfx950 with hipcc, in
parallel, and links them into ``libfgcg.so`` next to this file (the library
the binding loads).  Packed-FP32 instruction selection is disabled for every
HIP translation unit, and floating-point contraction is limited to single
expressions (results do not depend on how a template is instantiated).
Objects go to ``_build/`` beside the package.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfgcg.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("fgcg.hip", "fgcg3d.hip", "homog.hip", "noalloc.hip", "multiscale.hip")]

COMPILE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused per source expression only, so every
    # instantiation of a kernel template (rows per block, tiles) rounds alike
    "-ffp-contract=on",
    "-I" + os.path.join(ROOT, "include"),
]
LINK_FLAGS = ["--offload-arch=gfx950", "-shared", "-fPIC"]
NOISE = "is not a recognized feature for this target"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)


def build_library(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in SOURCES]
    cmds = [[hipcc()] + COMPILE_FLAGS + ["-c", s, "-o", o] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(len(cmds)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc()] + LINK_FLAGS + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
