"""Build libgps.so (HIP for gfx950) in the package directory.

    python -m paper_1509_00680_amd.build        # or build() from Python

Every source is compiled on each call; the objects go to _build/ beside the
sources, the library to paper_1509_00680_amd/libgps.so and the benchmark's
measurement kernels to paper_1509_00680_amd/libgps_micro.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgps.so")
SOURCES = ["gps_fft.hip", "gps_fft_fast.hip", "gps_ops.hip", "gps_cavity.hip", "gps_api.hip",
           "gps_server.hip"]
# measurement kernels of the benchmark (a library of their own, outside the C ABI)
MICRO_SOURCE = "gps_micro.hip"
MICRO_LIB = os.path.join(PKG, "libgps_micro.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
          # packed FP32 instructions are kept out of every kernel
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # x + 0.0 folds to x: the zero halves of padded transforms cost nothing
          "-fno-signed-zeros",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Wno-unused-command-line-argument"]


def _compile(src):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return out


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        objs = list(ex.map(_compile, SOURCES + [MICRO_SOURCE]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], MICRO_LIB)
    if verbose:
        print("built", LIB, "and", MICRO_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
