"""Build libsfw.so (HIP for gfx950) in-tree with hipcc: every source compiled to an object in
parallel (paper_2009_05473_amd/_build/), then linked."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsfw.so")
OBJ_DIR = os.path.join(PKG, "_build")
SOURCES = ["sfw_kernels.hip", "sfw_fft.hip", "sfw_fft_fixed.hip", "sfw_blur.hip", "sfw_api.cpp",
           "sfw_solver.cpp", "sfw_nnqp.cpp", "sfw_batch.cpp", "sfw_cnn.hip", "sfw_noalloc.hip",
           "sfw_nnqp_dev.hip"]
ARCH = "gfx950"
# hipcc's host pass does not know the packed-FP32 target feature; its warning is noise
NOISE = "is not a recognized feature for this target"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libsfw)")


def compile_command(src: str, obj: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # no packed-FP32 VALU instructions anywhere in the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-x", "hip", "-c", os.path.join(CSRC, src), "-I", INCLUDE, "-I", CSRC, "-o", obj]


def link_command(objs: list, out: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-pthread", "-o", out]


def command(out: str = LIB) -> list:
    """One hipcc line building the whole library (kept for reference; build() compiles the
    sources in parallel with the same flags)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-x", "hip", *srcs, "-I", INCLUDE, "-I", CSRC, "-pthread", "-o", out]


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in proc.stderr.splitlines() if NOISE not in l)
    return proc.returncode, err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link libsfw.so next to this file (always rebuilds)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [compile_command(s, o) for s, o in zip(SOURCES, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    for src, (rc, err) in zip(SOURCES, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src} ({rc}):\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    rc, err = _run(link_command(objs, tmp))
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
