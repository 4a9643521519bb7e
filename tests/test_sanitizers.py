"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: the library's
host sources (prime search, samplers, encoder, CRT, planner, wire format, argument checks) and the
C oracle are rebuilt with both sanitizers and the host-side test files run against those builds in
a child process with the sanitizer runtime preloaded. Any invalid access, leak-free misuse of the
heap or undefined operation aborts the child. The oracle's end-to-end tests at N = 2^14 are left
out to keep the run short (the same code runs at N = 2^12 and 2^13)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def test_host_code_under_sanitizers(tmp_path):
    from paper_2205_11935_amd import build as libbuild
    from oracle import build as orbuild
    lib = libbuild.build_sanitized(str(tmp_path / "lib"))
    olib = orbuild.build_sanitized(str(tmp_path / "oracle"))
    env = dict(os.environ)
    env.update({"CTL_LIB_PATH": lib, "CTL_ORACLE_LIB": olib, "LD_PRELOAD": libbuild.sanitizer_runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    files = ["tests/test_lib_host.py", "tests/test_wire_format.py", "tests/test_oracle_pins.py",
             "tests/test_oracle_cnn.py", "tests/test_oracle_properties.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not large and not end_to_end"] + files,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:] + r.stderr[-4000:])
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr
