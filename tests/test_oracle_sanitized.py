"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): tests/sanitize_driver.c is built together with oracle/eik_oracle.c
with both sanitizers (every report fatal) and runs every oracle entry point
on seeded random problems, including degenerate shapes and cell sides from 1
to beyond the grid.  The driver is a standalone executable, so no sanitizer
runtime has to be injected into the Python process."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
           os.path.join(ROOT, "tests", "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "eik_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), "40"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok")
