"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) and driven through every entry point on small cases by
tests/native/oracle_sanitized.c: no invalid access, leak or undefined
behaviour, and the exact invariants hold."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "oracle_san")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-ffp-contract=off", "-o", exe,
                               os.path.join(ROOT, "oracle", "vlasov_oracle.c"),
                               os.path.join(HERE, "native", "oracle_sanitized.c"), "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert out.returncode == 0, out.stdout + out.stderr
        assert out.stdout.strip().endswith("ok"), out.stdout
