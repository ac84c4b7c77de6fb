"""Build the HIP library (libtnlm.so) in-tree for gfx950 with hipcc.

Usage: python -m paper_1009_1351_amd.build [--jobs N]
Objects go to paper_1009_1351_amd/_build/, the shared library next to this
file. Every call recompiles (this is the "does it build" check).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtnlm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["api.hip", "proj.hip", "cgls.hip", "tnlm_reg.hip", "tnlm_reg_mfma.hip", "fbp.hip", "cnn.hip", "cnn_net.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(HERE, "..", "include"),
]

# The projector pair takes finite images and plane tables only: without NaN
# semantics its min/max need no quieting of their operands.
FILE_FLAGS = {"proj.hip": ["-fno-honor-nans"]}


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 4, verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    _build_capi_test(verbose)
    return LIB


def _build_capi_test(verbose: bool) -> None:
    """The C program of tests/capi, compiled as plain C against the header and
    linked to the in-tree library (it checks that the boundary is C)."""
    root = os.path.dirname(HERE)
    src = os.path.join(root, "tests", "capi", "solve_c.c")
    if not os.path.exists(src):
        return
    exe = os.path.join(root, "tests", "capi", "solve_c")
    cmd = ["gcc", "-O2", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(root, "include"), src, "-o", exe, "-L" + HERE, "-ltnlm",
           "-Wl,-rpath," + HERE, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C test program failed to build:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", exe)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
