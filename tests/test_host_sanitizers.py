"""CPU: the host-side paths of the C ABI (option validation, curve checks, expansion lengths,
profiling state, the no-device errors) built with AddressSanitizer and UndefinedBehaviorSanitizer
on the host code and run as a plain executable (tests/native/host_checks.cpp); any invalid memory
access, leak or undefined behaviour in the host code aborts it."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "native"))


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device paths")
def test_host_code_under_sanitizers():
    import build_sanitized
    exe = build_sanitized.build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
