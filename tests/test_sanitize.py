"""The C parts of the test reference (oracle/oracle.c) and of the input
generator (graphgen/graphgen.c) built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and run through a C driver
of oracle pins (tests/sanitize/oracle_checks.c): every check passes and no
sanitizer reports an error (the sanitizers abort on the first)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_and_generator_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_checks.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "graphgen", "graphgen.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "sanitize ok" in r.stdout, (r.returncode, r.stdout, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
