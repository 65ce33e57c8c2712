"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only), driven over small and empty shapes and malformed
inputs by oracle/sanitize_check.c, with the OpenMP passes at 1 and 4
threads.  Any invalid access or undefined operation fails the run."""

import os
import shutil
import subprocess

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    src = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "sanitize_check.c")]
    flags = [f for f in oracle.CFLAGS if f != "-O2"] + ["-O1", "-g", "-fno-omit-frame-pointer",
                                                       "-fsanitize=address,undefined",
                                                       "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", *flags, *src, "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passed" in r.stdout
