"""Build the AIRPF CPU oracle shared library (oracle/liborc.so) with gcc.

TEST INFRASTRUCTURE ONLY: the oracle is a checker, never part of the product
path.  Built with -ffp-contract=off so that every fused multiply-add in the
sources is an explicit fma() call and nothing else is contracted.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_math.c", "orc_rng.c", "orc_models.c", "orc_airpf.c", "orc_bpf.c"]
OUT = os.path.join(HERE, "liborc.so")
FLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc", *FLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
