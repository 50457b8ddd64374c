"""The decoder's binary64 digit arithmetic (kernels_common.h: split_word, digit_off), compiled
for the host and checked against exact integer division: every base 2..2^16 + 1 with edge and
random words, and random bases of u32 data up to 2^32."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_split_and_digits_match_integer_division(tmp_path):
    exe = str(tmp_path / "split_check")
    src = os.path.join(ROOT, "tests", "host", "split_check.cpp")
    inc = os.path.join(ROOT, "paper_1805_01844_amd", "csrc")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", inc,
                           "-o", exe, src], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], stdout=subprocess.PIPE, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
