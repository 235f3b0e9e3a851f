"""Build libc0ip.so in-tree for gfx950 (hipcc for the HIP sources, g++ for
the host set-up and for the generator of the reference-coefficient header).  Usage: ``python -m paper_2412_05082_amd.build``."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libc0ip.so")

HIP_SOURCES = ["kernels2d.hip", "op2d.hip", "op2d_avs64.hip", "op2d_avs32.hip", "op3d.hip", "smooth3d.hip", "kernels3d.hip", "kernels_common.hip", "api.hip", "batch.hip", "vtail.hip", "krylov_cg.hip", "mvs3d.hip"]
CXX_SOURCES = ["setup.cpp"]
ARCH = os.environ.get("C0IP_OFFLOAD_ARCH", "gfx950")
# packed FP32 instructions are kept out of every code object
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}", f"-I{BUILD}"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    # generated header: reference 1D coefficient rows (compile-time constants of the 3D operator)
    gen = os.path.join(BUILD, "gen_refcoef")
    _run(["g++", "-O2", "-std=c++17", f"-I{CSRC}", os.path.join(CSRC, "gen_refcoef.cpp"),
          os.path.join(CSRC, "setup.cpp"), "-o", gen])
    _run([gen, os.path.join(BUILD, "refcoef.h")])
    cmds = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", f"-I{CSRC}", "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([hipcc, *HIP_FLAGS, "-shared", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
