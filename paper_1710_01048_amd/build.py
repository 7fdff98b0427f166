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


def _run_all(cmds, verbose):
    """Runs the commands side by side; raises if any fails (after all have ended)."""
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, pr in procs if pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])


def build(verbose=False):
    """Compile every source and link paper_1710_01048_amd/libwqa.so (always rebuilds)."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    # the kernels source once per part (forward, products, FP32 and FP64 adjoint), the
    # blocked 3D products, the host code and the probes: independent compilations, run
    # side by side
    jobs = []
    k_objs = []
    for part in range(4):
        obj = os.path.join(BUILD, f"wqa_kernels_{part}.o")
        k_objs.append(obj)
        jobs.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, f"-DWQA_PART={part}",
                     "-Wno-unneeded-internal-declaration", "-Wno-unused-function", "-c",
                     os.path.join(CSRC, "wqa_kernels.hip"), "-o", obj])
    p_obj = os.path.join(BUILD, "wqa_products.o")
    k_objs.append(p_obj)
    jobs.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-c",
                 os.path.join(CSRC, "wqa_products.hip"), "-o", p_obj])
    h_obj = os.path.join(BUILD, "wqa_host.o")
    jobs.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-c",
                 os.path.join(CSRC, "wqa_host.cpp"), "-o", h_obj])
    ptmp = PROBES + ".tmp%d" % os.getpid()
    jobs.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-shared",
                 os.path.join(CSRC, "wqa_probes.hip"), "-o", ptmp])
    _run_all(jobs, verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *k_objs, h_obj], verbose)
    os.replace(tmp, LIB)
    # the memory-pattern probes (measurement only; the bench loads them)
    os.replace(ptmp, PROBES)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
