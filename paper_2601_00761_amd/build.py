"""Compile libpauliwht.so for gfx950 in-tree with hipcc.

Every translation unit is HIP C++; the shared library exports only the C ABI
declared in include/pauliwht.h.  Packed FP32 instructions are disabled
(-packed-fp32-ops) for all device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["fwht.hip", "state.hip", "sample.hip", "made.hip", "clifford.hip", "api.hip", "noalloc.hip"]
LIB = os.path.join(HERE, "libpauliwht.so")
ARCH = os.environ.get("PW_OFFLOAD_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _compile(src):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    build_example(verbose)
    return LIB


EXAMPLE_SRC = os.path.join(HERE, "examples", "exact_c.c")
EXAMPLE_BIN = os.path.join(HERE, "examples", "exact_c")
EXAMPLE_LIB = os.path.join(HERE, "examples", "libexact_c.so")


def build_example(verbose=False):
    """The plain-C client of the ABI (gcc, the header and the HIP runtime only), as a
    program and as a shared object without main (loaded in-process by the tests)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    common = ["gcc", "-O2", "-std=c11", "-Wall", "-I" + os.path.join(ROOT, "include"),
              "-I" + os.path.join(rocm, "include"), EXAMPLE_SRC]
    link = ["-L" + HERE, "-lpauliwht", "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
            "-Wl,-rpath,$ORIGIN/..:" + os.path.join(rocm, "lib")]
    for cmd in (common + ["-o", EXAMPLE_BIN] + link,
                common + ["-DEXACT_C_NO_MAIN", "-fPIC", "-shared", "-o", EXAMPLE_LIB] + link):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("example build failed:\n" + r.stderr)
    if verbose:
        print("built", EXAMPLE_BIN, EXAMPLE_LIB)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
