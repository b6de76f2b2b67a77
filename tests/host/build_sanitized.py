"""Host-sanitizer build of libsfw for the CPU tests (tests/test_host_sanitized.py).

libsfw_sanitized.so: the library's host C++ sources (workspace, argument validation, solver,
NNQP, batch) compiled by g++ with AddressSanitizer and UndefinedBehaviorSanitizer, linked with
the device sources' objects of the last regular build (paper_2009_05473_amd/build.py, compiled
without sanitizers). nnqp_check: tests/host/nnqp_check.cpp with the library's NNQP, sanitized.
Load the library with the sanitizer runtimes preloaded (see the test).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2009_05473_amd import build as B  # noqa: E402

HOST_SOURCES = [s for s in B.SOURCES if s.endswith(".cpp")]
SANITIZE = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
OUT = os.path.join(B.OBJ_DIR, "sanitized")


def rocm_root():
    return os.path.dirname(os.path.dirname(os.path.realpath(B.hipcc())))


def gxx(args):
    r = subprocess.run(["g++", *args], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed:\n" + r.stderr[-4000:])


def host_flags():
    return ["-std=c++17", "-O1", "-g", "-fPIC", *SANITIZE, "-D__HIP_PLATFORM_AMD__", "-I",
            os.path.join(rocm_root(), "include"), "-I", B.INCLUDE, "-I", B.CSRC]


def build_library():
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src in B.SOURCES:
        if src in HOST_SOURCES:
            obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
            gxx([*host_flags(), "-c", os.path.join(B.CSRC, src), "-o", obj])
        else:
            obj = os.path.join(B.OBJ_DIR, os.path.splitext(src)[0] + ".o")
            if not os.path.exists(obj):
                raise RuntimeError(f"{obj} missing: build the library first")
        objs.append(obj)
    lib = os.path.join(rocm_root(), "lib")
    out = os.path.join(OUT, "libsfw_sanitized.so")
    gxx(["-shared", "-fPIC", *SANITIZE, *objs, "-L", lib, "-lamdhip64", f"-Wl,-rpath,{lib}",
         "-pthread", "-o", out])
    return out


def build_nnqp_check():
    os.makedirs(OUT, exist_ok=True)
    out = os.path.join(OUT, "nnqp_check")
    gxx([*host_flags(), os.path.join(HERE, "nnqp_check.cpp"),
         os.path.join(B.CSRC, "sfw_nnqp.cpp"), "-o", out])
    return out


def runtimes():
    """Paths of the ASan and UBSan runtimes to preload into an uninstrumented Python."""
    paths = []
    for name in ("libasan.so", "libubsan.so"):
        r = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
        paths.append(r.stdout.strip())
    return paths


if __name__ == "__main__":
    print(build_library())
    print(build_nnqp_check())
