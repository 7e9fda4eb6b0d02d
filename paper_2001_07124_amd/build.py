"""Build librhosvd.so (the HIP library behind include/rhosvd.h) for gfx950.

    python -m paper_2001_07124_amd.build        # or build_library() from Python

The library is compiled in-tree next to this file with hipcc.  Every HIP
source is compiled with the packed-FP32 target feature turned off.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librhosvd.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "kernels_wave.hip", "kernels_small.hip", "rhosvd_api.hip")]
ARCH = os.environ.get("RHOSVD_ARCH", "gfx950")


def hipcc_path():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build_library(verbose=False):
    cmd = [hipcc_path(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build librhosvd.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
