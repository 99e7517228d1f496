"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): ``oracle/oracle.c`` and ``tests/oracle_sanitize_main.c`` are
built into one executable with gcc and run; every exported oracle function is
called on small inputs and edge cases, and any sanitizer report (out-of-bounds
access, leak, signed overflow, bad shift, ...) or failed identity fails the
test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(ROOT, "oracle", "oracle.c")]

# same code-generation options as the oracle library (one rounding per
# operation), plus the sanitizers; the host compiler only, no device code
SAN_FLAGS = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    build = subprocess.run(["gcc", *SAN_FLAGS, *SRC, "-o", exe, "-lm"], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all checks passed" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr
