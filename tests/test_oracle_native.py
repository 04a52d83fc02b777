"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
small C++ driver calls every entry point (tests/native/), built with g++ (the
oracle is plain host C++) and run in a subprocess that stops at the first
report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    srcs = [os.path.join(ROOT, "oracle", "band_oracle.cpp"),
            os.path.join(HERE, "native", "oracle_sanitize_driver.cpp")]
    subprocess.run(["g++", *flags, *srcs, "-o", str(exe)], check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().startswith("ok")
