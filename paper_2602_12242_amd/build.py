"""Builds libmagx.so (gfx950) in-tree with hipcc.

    python -m paper_2602_12242_amd.build          # or build() from Python

Every HIP source and the C-ABI host file are compiled in one hipcc call.
Packed-FP32 instructions are disabled for the device code.  The sign of a
zero result is not significant anywhere in the library, so x + 0 may fold to
x (the zero-padded halves of the first FFT passes then cost no arithmetic).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libmagx.so")
SOURCES = ["magx_api.cpp", "tensor.hip", "conv.hip", "pencil.hip", "mri.hip"]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose=False):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-fgpu-rdc", "--hip-link",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-fno-signed-zeros",
           "-Wno-unused-command-line-argument",
           "-I", INCLUDE, "-o", tmp] + [("-x", "hip", s) if s.endswith(".hip") else ("-x", "hip", s) for s in srcs]
    flat = []
    for c in cmd:
        if isinstance(c, tuple):
            flat.extend(c)
        else:
            flat.append(c)
    if verbose:
        print(" ".join(flat), flush=True)
    res = subprocess.run(flat, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmagx.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
