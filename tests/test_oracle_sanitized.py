"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven over small inputs and edge cases by
tests/csrc/oracle_sanitized_driver.c: no invalid access or undefined
operation, and the functions agree with one another (CPU only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
           os.path.join(ROOT, "tests", "csrc", "oracle_sanitized_driver.c"),
           os.path.join(ROOT, "oracle", "symba_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    # a library preloaded by the environment may come before the sanitizer runtime
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and r.stdout.strip().endswith("ok"), r.stderr[-2000:]
