"""Build paper_1209_3516_amd/libfmm.so: host C++ (g++) + gfx950 kernels (hipcc).

Host code (tree, traversal, work plan, C interface) is compiled without FMA
contraction or fast-math so that keys, centres, radii and the acceptance test
are reproducible bit for bit.  Device code is compiled for gfx950 only, with
packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["tree.cpp", "traverse.cpp", "plan.cpp", "shard.cpp", "m2l_plan.cpp", "api.cpp"]
DEVICE_SOURCES = ["p2p.hip", "far.hip", "misc.hip", "tree_gpu.hip", "plan_gpu.hip", "noalloc.hip",
                  "m2l_mfma.hip"]
# Sources whose FP64 arithmetic must match the host bit for bit (no FMA contraction).
EXACT_SOURCES = {"tree_gpu.hip"}

HOST_FLAGS = ["-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
              "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
              "-I" + CSRC, "-I" + os.path.join(ROCM, "include")]
DEVICE_FLAGS = ["-std=c++20", "-O3", "-fPIC", "--offload-arch=gfx950", "-fbracket-depth=4096",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        extra = ["-ffp-contract=off"] if src in EXACT_SOURCES else []
        cmd = [os.path.join(ROCM, "bin", "hipcc")] + DEVICE_FLAGS + extra + [
            "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("compile failed: " + " ".join(failed[0]))
    link = ["g++", "-shared", "-fopenmp", "-o", LIB + ".tmp"] + objs + [
        "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    _run(link, verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
