"""Build the gfx950 shared library `lib/liblamino.so` in-tree with hipcc
(plus `lib/libcopycalib.so`, the counter-calibration copies, and the
host self-test of the kernels' index logic).

Usage: python -m paper_2401_11101_amd.build  (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "liblamino.so")
SELFTEST = os.path.join(LIBDIR, "lamino_selftest_host")
CALIB = os.path.join(LIBDIR, "libcopycalib.so")

SOURCES = ["lamino_api.cpp", "lamino_kernels.hip", "lamino_tv.hip", "lamino_direct.hip",
           "lamino_scratch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    # packed fp32 VALU ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=False):
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include")]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # copy kernels that calibrate the HBM byte counters (measurement only)
    tmp = CALIB + ".tmp"
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, "copy_calib.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CALIB)
    # host-only checks of the kernels' index logic
    tmp = SELFTEST + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "selftest_host.cpp"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SELFTEST)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
