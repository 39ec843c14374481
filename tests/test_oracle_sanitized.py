"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(plain gcc, host code only): every message in an exact-size heap block, so
a read past a message's end, an out-of-range shift (the remainder's rotate by
r, 1 <= r <= 31) or a signed overflow stops the run.  The driver,
tests/oracle_sanitized_main.c, also checks streaming = one-shot, the output
prefix structure and the threaded batch driver."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitized_main.c"), os.path.join(ROOT, "oracle", "hh_oracle.c"),
           "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    if build.returncode != 0 and ("asan" in build.stderr or "ubsan" in build.stderr):
        pytest.skip("sanitizer runtime not installed: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    if run.returncode != 0 and "does not come first in initial library list" in run.stderr:
        pytest.skip("the environment preloads a library ahead of the sanitizer runtime")
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr, run.stderr[-4000:]
    assert "all checks passed" in run.stdout
