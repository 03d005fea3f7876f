"""The CPU oracle under AddressSanitizer (with leak detection) and
UndefinedBehaviorSanitizer: tests/sanitize_driver.c calls every entry point on
small, ragged and empty problems with every optional output and both rules;
any out-of-bounds access, use after free, leak or undefined operation aborts
the run.  Host code only, built with gcc."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "orc_san"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
           "-Wno-unknown-pragmas", "-o", str(exe),
           os.path.join(ROOT, "tests", "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "preprocess_oracle.c"), "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "sanitize" in (b.stderr or ""):
        pytest.skip("gcc has no sanitizer runtime here: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
