"""Build the HIP library libh2bem.so for gfx950 (in-tree, no JIT cache).

    python paper_2001_05523_amd/csrc/build_lib.py

Runs as a plain script (it does not import the package, whose import loads
the library).
"""
import concurrent.futures
import os
import subprocess
import sys

CSRC = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(CSRC)
ROOT = os.path.dirname(PKG)
OUT_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(OUT_DIR, "libh2bem.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["host_trees.cpp", "host_linalg.cpp", "kernels.hip", "kernels_mrhs.hip", "op.hip", "recompress.hip", "batch.hip", "batch_merged.hip", "symnear.hip", "symcpl.hip", "krylov.hip", "gca.hip", "gca_host.cpp", "recompute.hip", "transform.hip", "hmatrix.cpp", "hchol.hip", "capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# every translation unit goes through hipcc so device code (if any) gets the
# same target features; packed-fp32 instructions are disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") or src.endswith(".cpp") else []
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
