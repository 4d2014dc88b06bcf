"""Build libmbo.so (HIP kernels for gfx950 + host runtime + C ABI) in-tree.

    python -m paper_1711_01365_amd.build

hipcc cross-compiles for gfx950 without a GPU.  Packed-FP32 instructions are
disabled for device code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmbo.so")
SOURCES = ["mbo_row_f32.hip", "mbo_row_f64.hip", "mbo_col_f32.hip", "mbo_col_f64.hip",
           "mbo_vprow_f32.hip", "mbo_vprow_f64.hip", "mbo_volume.hip", "mbo_relaxrow_f32.hip",
           "mbo_relaxrow_f64.hip", "mbo_misc.hip", "mbo_fast_f32.hip", "mbo_fast_f64.hip", "mbo_surface.hip", "mbo_surfvol.hip",
           "mbo_static.hip", "mbo_api.cpp"]
HEADERS = ["mbo_device.hpp", "mbo_kernels.hpp", "mbo_internal.hpp", "mbo_volume.hpp", "mbo_fast.hpp",
           "mbo_fast_launch.hpp"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libmbo)")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def _compile(args):
    cmd, verbose = args
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, r.returncode, r.stdout + r.stderr


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every translation unit (in parallel) and link libmbo.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    work, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        work.append(([cc] + flags() + lang + ["-c", os.path.join(CSRC, src), "-o", obj], verbose))
        objs.append(obj)
    jobs = jobs or min(len(work), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, rc, out in ex.map(_compile, work):
            if rc != 0:
                sys.stderr.write(out)
                raise RuntimeError("compilation failed: " + " ".join(cmd))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
