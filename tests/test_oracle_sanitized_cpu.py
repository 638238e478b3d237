"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_check.c calls every function the oracle exports on small
inputs with exactly sized heap buffers and checks invariants that hold for
any input (permutations, a symmetric deposit totalling 2 n sum(q), the
optimum no longer than a constructed tour).  It is built here with gcc and
both sanitizers, errors fatal, and must exit 0 with no report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_check")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-o", exe,
           os.path.join(ORACLE, "sanitize_check.c"), os.path.join(ORACLE, "aco_oracle.c"),
           os.path.join(ORACLE, "mlp_oracle.c"), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "sanitize_check: ok" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr
    assert "runtime error" not in run.stderr
