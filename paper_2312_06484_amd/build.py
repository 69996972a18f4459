"""Build the AIRPF HIP library in-tree: paper_2312_06484_amd/libairpf.so.

hipcc for gfx950 only.  -ffp-contract=off keeps every fused multiply-add an
explicit fma() (the arithmetic contract with the CPU checker), and packed
FP32 instructions are switched off.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libairpf.so")
SOURCES = ["forward.hip", "score.hip", "capi.hip"]
ARCH = "gfx950"


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False, out: str = OUT) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *flags(), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
