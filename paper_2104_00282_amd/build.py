"""Build libresalloc.so (gfx950 HIP kernels + host runtime) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libresalloc.so")
SOURCES = ["kernels.hip", "runtime.hip", "mlp.hip", "probe.hip", "loop.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(verbose: bool = False, extra=()) -> str:
    """Compile every HIP source into paper_2104_00282_amd/libresalloc.so."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libresalloc.so")
    noise = [l for l in (res.stdout + res.stderr).splitlines()
             if l.strip() and "packed-fp32-ops" not in l]
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")
    os.replace(tmp, LIB)
    return LIB


C_DEMO_SRC = os.path.join(ROOT, "tests", "c_consumer", "solve_demo.c")
C_DEMO = os.path.join(ROOT, "tests", "c_consumer", "solve_demo")


def build_c_consumer(verbose: bool = False) -> str:
    """Compile the plain C consumer of the C ABI used by the GPU tests
    (gcc, linked against the in-tree libresalloc.so and the HIP runtime)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = C_DEMO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           C_DEMO_SRC, "-o", tmp, "-L", HERE, "-lresalloc", "-L", os.path.join(rocm, "lib"),
           "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_2104_00282_amd",
           "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("gcc failed building the C consumer")
    os.replace(tmp, C_DEMO)
    return C_DEMO


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_c_consumer(verbose=True))
