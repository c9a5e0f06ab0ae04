"""Build libtomo.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1604_02292_amd.build
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtomo.so")

SOURCES = ["tomo_kernels.hip", "tomo_plan.cpp", "tomo_capi.cpp", "tomo_serve.cpp", "tomo_local.cpp",
           "tomo_noalloc.hip", "tomo_probe.hip"]

# Packed FP32 instructions are disabled for all device code on this target.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, verbose):
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    if src.endswith(".hip"):
        cmd = [_hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + ["-x", "hip"] + DEVICE_FLAGS
    else:
        # host-only runtime code: plain C++ against the HIP runtime headers
        cmd = ["g++", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + [
            "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-o", tmp] + objs + DEVICE_FLAGS + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
