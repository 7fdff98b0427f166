"""Builds libwqa.so (host C ABI + gfx950 HIP kernels) and libwqa_probes.so (memory-pattern
probes for the benchmark) in-tree with hipcc.

    python paper_1710_01048_amd/build.py [-q]

Run as a script (or loaded by file path, as __graft_entry__.build() does): importing it
through the package would load the library it is about to build.

All HIP code is compiled for gfx950 only, with packed-FP32 instruction selection
turned off (-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwqa.so")
PROBES = os.path.join(HERE, "libwqa_probes.so")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm required to build libwqa.so)")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False):
    """Compile every source and link paper_1710_01048_amd/libwqa.so (always rebuilds)."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    k_obj = os.path.join(BUILD, "wqa_kernels.o")
    h_obj = os.path.join(BUILD, "wqa_host.o")
    _run([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-c",
          os.path.join(CSRC, "wqa_kernels.hip"), "-o", k_obj], verbose)
    _run([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-c",
          os.path.join(CSRC, "wqa_host.cpp"), "-o", h_obj], verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, k_obj, h_obj], verbose)
    os.replace(tmp, LIB)
    # the memory-pattern probes (measurement only; the bench loads them)
    tmp = PROBES + ".tmp%d" % os.getpid()
    _run([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-shared",
          os.path.join(CSRC, "wqa_probes.hip"), "-o", tmp], verbose)
    os.replace(tmp, PROBES)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
