"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/oracle_sanitize.c is compiled together with oracle/lfo.c by gcc with both
sanitizers, no recovery, and the oracle's own numeric flags (no FMA contraction); it runs
closed-form pins, naive-vs-factored equality with the state re-checked after every queue,
and every other oracle entry point once.  Any sanitizer report aborts the driver.
(ThreadSanitizer is not used: libgomp is not instrumented, so it reports its own
synchronisation as races.)
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ROOT, "tests", "oracle_sanitize.c"), os.path.join(ROOT, "oracle", "lfo.c"), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize ok" in r.stdout
