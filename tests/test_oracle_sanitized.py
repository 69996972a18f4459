"""The CPU oracle's C sources built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and run through every entry
point by oracle/orc_sanitize_main.c: out-of-bounds accesses, leaks,
misaligned or overflowing operations in its manual array indexing abort the
run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    srcs = [os.path.join(ORC, f) for f in ["orc_math.c", "orc_rng.c", "orc_models.c", "orc_airpf.c", "orc_bpf.c",
                                           "orc_sanitize_main.c"]]
    with tempfile.TemporaryDirectory(prefix="orc_san_") as d:
        exe = os.path.join(d, "orc_san")
        cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe, *srcs, "-lm"]
        subprocess.run(cmd, check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
        assert "ok" in r.stdout
