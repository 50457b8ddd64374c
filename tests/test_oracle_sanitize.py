"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (gcc): round trips of
every element width, block length and variant kind, and decoding of damaged streams, with every
buffer at its exact size (tests/host/oracle_sanitize.c). Host code only: no GPU is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_and_ubsan(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = [cc, "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, os.path.join(ROOT, "tests", "host", "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "pcomp_oracle.c"), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600, env=env)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout[-4000:]
