"""The device's FP64 -> BF16 rounding, compiled for the host and checked
against a plain definition of round-to-nearest-even (tests/native)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_bf16_rounding_is_round_to_nearest_even():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "bf16")
        subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-o", exe,
                               os.path.join(HERE, "native", "bf16_rounding.cpp")],
                              stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0, out.stdout
        assert out.stdout.strip().endswith("0 of 14000000 mismatched")
