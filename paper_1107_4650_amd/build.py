"""Build libdirac.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed FP32
instructions disabled, and linked into one shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "lib", "libdirac.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["dirac_sweep2d_f32_hi.hip", "dirac_sweep2d_f64_hi.hip", "dirac_sweep2d_f32_lo.hip",
           "dirac_sweep2d_f64_lo.hip", "dirac_sweep2d_strang.hip", "dirac_batch.hip",
           "dirac_sweep3d.hip", "dirac_adjoint.hip", "dirac_plan.hip", "dirac_sweep.hip",
           "dirac_reduce.hip", "dirac_sweep2d_obs.hip", "dirac_sweep1d_deep.hip"]
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(ROOT, "include", "libdirac.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(
            os.path.getmtime(os.path.join(CSRC, src)), _headers_mtime()):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile all sources and link libdirac.so; returns its path.  With
    incremental=True, objects newer than their source and every header are
    reused."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), SOURCES))
    tmp = OUT + ".tmp"
    # roctx: the named host ranges of the entry points (rocprofv3 --marker-trace)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
           "-L" + ROCM_LIB, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + ROCM_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    import sys
    build(verbose=True, incremental="--incremental" in sys.argv)
