"""The oracle built with the address and undefined-behaviour sanitizers
(g++, host code only) and run by a small C++ driver that calls every one of
its functions on lattices of 3 to 17 nodes, for every equilibrium kind with
and without the source, and on rejected arguments (no GPU)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitized")
        flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-g", "-O1", "-std=c++17",
                 "-ffp-contract=off"]
        subprocess.run(["g++", *flags, "-I", os.path.join(ROOT, "oracle"),
                        os.path.join(ROOT, "oracle", "lbm_oracle.cpp"),
                        os.path.join(ROOT, "tests", "oracle_sanitize_driver.cpp"),
                        "-o", exe], check=True)
        env = dict(os.environ,
                   ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env,
                           timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "runtime error" not in r.stderr, r.stderr
        assert "0 failures" in r.stdout
