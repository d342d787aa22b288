"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sancheck.c drives every storage format through encode/decode, the
SpMV, the dot, block-Jacobi set-up and restarted CB-GMRES with every format,
preconditioner and variant bit (debug outputs on and off, b = 0, n = 1) on
small seeded systems.  It is compiled here with oracle.c by gcc with
-fsanitize=address,undefined (host code; the oracle has no GPU code) and
run; any sanitizer report, leak or unexpected status fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "sancheck.c")]


def test_oracle_clean_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sancheck")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror", "-fopenmp",
           "-ffp-contract=off", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", *SRC, "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "LeakSanitizer" not in r.stderr, r.stderr
    assert r.stdout.rstrip().endswith("PASSED: 0 failure(s)")
    assert r.stdout.count("\nok   gmres") == 100
