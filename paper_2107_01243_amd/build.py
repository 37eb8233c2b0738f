"""Build libsem.so (HIP for gfx950) in-tree.

ax_kernels.hip and schwarz_kernels.hip are compiled once per supported lx (2..16)
so the instantiations build in parallel; the objects are linked with the vector kernels, the host
setup code and the C ABI into paper_2107_01243_amd/libsem.so.

Usage: python paper_2107_01243_amd/build.py [--jobs N]   (run by path: importing the
package would load the library being built)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libsem.so")
BUILD = os.path.join(ROOT, "_build", "libsem")
ARCH = "gfx950"
LX_RANGE = range(2, 17)

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU instructions.
DEVICE_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I", CSRC, "-I", INCLUDE]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return cmd[-1]


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    steps = []
    for lx in LX_RANGE:
        obj = os.path.join(BUILD, f"ax_lx{lx}.o")
        steps.append([HIPCC, *DEVICE_FLAGS, f"-DSEM_LX={lx}", "-c",
                      os.path.join(CSRC, "ax_kernels.hip"), "-o", obj])
        steps.append([HIPCC, *DEVICE_FLAGS, f"-DSEM_LX={lx}", "-c",
                      os.path.join(CSRC, "schwarz_kernels.hip"), "-o", os.path.join(BUILD, f"schwarz_lx{lx}.o")])
    for src in ("vec_kernels.hip", "sem_noalloc.hip", "sem_api.cpp", "sem_cg.cpp", "sem_proj.cpp",
                "sem_gmres.cpp", "host_setup.cpp"):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        steps.append([HIPCC, *DEVICE_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_run, steps))
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
