"""Build step for libnq.so (gfx950): hipcc compiles every source under csrc/.

Usage:  python -m paper_2511_12009_amd.build [--asm DIR]
--asm DIR additionally writes the gfx950 assembly of every .hip source to DIR.
"""
import argparse
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libnq.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Marker ranges (nq_trace.h) come from the profiler SDK's roctx library.
ROCM_LIB = "/opt/rocm/lib"
# Packed FP32 instructions are kept out of every code object.  Loops start on
# a 64-byte instruction-cache line: the DFS step loop is 192 bytes, three lines
# when aligned; where it started 4 bytes before a line boundary the N = 20
# count ran 2 % slower.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-falign-loops=64"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          f"--offload-arch={ARCH}", "-I", os.path.join(os.path.dirname(HERE), "include")]

SOURCES = ["nq_frontier.cpp", "nq_dfs.hip", "nq_expand.hip", "nq_api.cpp", "nq_batch.cpp", "nq_tune.cpp",
           "nq_serve.cpp", "nq_noalloc.hip", "nq_ubench.hip", "nq_perm.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _compile_one(src, verbose):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    _run([HIPCC] + COMMON + DEVICE_FLAGS + lang + ["-c", path, "-o", obj], verbose)
    return obj


def build(verbose: bool = False, asm_dir: str = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile_one(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread"] + objs +
         ["-L", ROCM_LIB, f"-Wl,-rpath,{ROCM_LIB}", "-lrocprofiler-sdk-roctx", "-o", tmp], verbose)
    os.replace(tmp, LIB)
    if asm_dir:
        os.makedirs(asm_dir, exist_ok=True)
        for src in SOURCES:
            if src.endswith(".hip"):
                out = os.path.join(asm_dir, os.path.splitext(src)[0] + f"-{ARCH}.s")
                _run([HIPCC] + COMMON + DEVICE_FLAGS + ["-x", "hip", "--cuda-device-only", "-S",
                                                        os.path.join(CSRC, src), "-o", out],
                     verbose)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", default=None)
    ap.add_argument("-q", action="store_true")
    a = ap.parse_args()
    print(build(verbose=not a.q, asm_dir=a.asm))
    sys.exit(0)
