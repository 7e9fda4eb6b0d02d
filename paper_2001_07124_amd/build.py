"""Build librhosvd.so (the HIP library behind include/rhosvd.h) for gfx950.

    python -m paper_2001_07124_amd.build        # or build_library() from Python

Each HIP source is compiled to an object in `_build/` next to this file (in
parallel), then linked in-tree.  Every source is compiled with the packed-FP32
target feature turned off.  The small dense kernels additionally ask the
backend to keep matrix-core accumulators in ordinary VGPRs: their
accumulators otherwise round-trip through AGPRs on every step of the loops.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librhosvd.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("RHOSVD_ARCH", "gfx950")
# source -> extra flags
SOURCES = {
    "kernels.hip": [],
    "kernels_wave.hip": [],
    "kernels_col.hip": [],
    "kernels_small.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "kernels_resid.hip": [],
    "kernels_trunc.hip": [],
    "kernels_allmode.hip": [],
    "kernels_batch.hip": [],
    "server.hip": [],
    "noalloc.hip": [],
    "rhosvd_api.hip": [],
}


def hipcc_path():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _common_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def _newest_header():
    paths = [os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))
             if f.endswith((".hpp", ".h"))]
    paths += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(p) for p in paths)


def _compile(hipcc, src, extra, verbose, incremental=False):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    srcp = os.path.join(HERE, "csrc", src)
    if incremental and os.path.exists(obj):
        if os.path.getmtime(obj) > max(os.path.getmtime(srcp), _newest_header()):
            return obj, None
    cmd = [hipcc, *_common_flags(), *extra, "-c", srcp, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        return obj, res.stdout + res.stderr
    return obj, None


def build_library(verbose=False, incremental=False):
    """Compile every source (incremental=True skips objects newer than their
    source and every header) and link librhosvd.so in-tree."""
    hipcc = hipcc_path()
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")) or 1)
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        results = list(pool.map(lambda kv: _compile(hipcc, kv[0], kv[1], verbose, incremental),
                                SOURCES.items()))
    errors = [err for _, err in results if err]
    if errors:
        sys.stderr.write("\n".join(errors))
        raise RuntimeError("hipcc failed to build librhosvd.so")
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *[o for o, _ in results],
           "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link librhosvd.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True, incremental="--incremental" in sys.argv))
