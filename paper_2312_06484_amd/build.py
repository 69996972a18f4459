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
SOURCES = ["forward.hip", "forward_models_1d.hip", "forward_models_lgd23.hip", "forward_models_lgd4.hip",
           "forward_models_lgd8.hip", "forward_models_bin.hip", "score.hip", "capi.hip"]
ARCH = "gfx950"


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def link_flags():
    """Libraries of the link: the ROCm tracer's range markers (roctx)."""
    return ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False, out: str = OUT) -> str:
    """Compile each source to an object (in parallel), then link."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp%d" % os.getpid()
    compile_flags = [f for f in flags() if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="airpf_build_") as d:
        objs = [os.path.join(d, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[hipcc(), *compile_flags, "-c", "-o", o, s] for s, o in zip(srcs, objs)]
        cmds.append([hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs, *link_flags()])
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
            for r in ex.map(lambda c: subprocess.run(c), cmds[:-1]):
                if r.returncode != 0:
                    raise subprocess.CalledProcessError(r.returncode, r.args)
        subprocess.run(cmds[-1], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
