"""Builds the in-tree native libraries.

  libqfuse.so            HIP kernels + host planner + C-ABI (hipcc, gfx950)
  libqfuse_plancheck.so  test-only CPU execution of the planner's programs (g++)

Every HIP source is compiled for gfx950 with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libqfuse.so")
PLANCHECK = os.path.join(PKG, "libqfuse_plancheck.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-Wno-unused-value"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build failed: {' '.join(cmd)}")


HIP_SOURCES = ("plan.cpp", "qfuse.hip", "batch.hip")


def build_hip(out: str = LIB) -> str:
    """Compiles every source to an object in parallel, then links the library."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIP_FLAGS if f != "-shared"]
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append((obj, [HIPCC, *compile_flags, f"-I{INCLUDE}", f"-I{CSRC}", "-c", os.path.join(CSRC, src),
                           "-o", obj]))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, cmd) for _, cmd in jobs]:
            f.result()
    tmp = out + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs], "-o", tmp])
    os.replace(tmp, out)
    return out


def build_plancheck(out: str = PLANCHECK) -> str:
    srcs = [os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "plancheck.cpp")]
    tmp = out + ".tmp"
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", f"-I{INCLUDE}", f"-I{CSRC}", *srcs, "-o", tmp])
    os.replace(tmp, out)
    return out


def build_all() -> None:
    build_hip()
    build_plancheck()


if __name__ == "__main__":
    build_all()
