"""Build the gfx950 HIP libraries in place (hipcc, no JIT cache): ``libcvetl.so``
and the checking build ``libcvetl_debug.so`` (``-DCVETL_DEBUG``: checker kernels
after each stage, see cv_debug_flags in the header).

Every HIP source is compiled for gfx950 only, with IEEE double division and
no floating-point contraction (``-ffp-contract=off``) so that kinematics and
grid binning evaluate exactly the expressions written in the kernels, and with
packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcvetl.so")
DEBUG_LIB = os.path.join(PKG, "libcvetl_debug.so")  # the checking build (CVETL_DEBUG)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(job) -> str:
    src, debug = job
    obj = os.path.join(BUILD, ("debug_" if debug else "") + os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DCVETL_DEBUG"] if debug else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Both libraries: libcvetl.so and the checking build libcvetl_debug.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = [(src, False) for src in srcs] + [(src, True) for src in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(_compile, jobs))
    _link(objs[:len(srcs)], LIB)
    _link(objs[len(srcs):], DEBUG_LIB)
    if verbose:
        print(f"built {LIB} and {DEBUG_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
