"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only).

``tests/helpers/orc_sanitize.c`` includes ``oracle/orc.c`` and calls every exported
function on small meshes (degrees 1-3, every flag combination the tests use, a degenerate
3 x 1 x 2 mesh).  It is compiled with gcc and both sanitizers, without OpenMP, and any
finding aborts the run with a non-zero status.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "helpers", "orc_sanitize.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = os.path.join(tmp_path, "orc_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           SRC, "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    assert "oracle sanitizer run: ok" in res.stdout
