"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
oracle/sanitize_check.cpp drives every oracle entry point on empty, tiny,
colliding and edge-address inputs and checks the routes against each other
and against closed forms; built with g++ and the sanitizers, any out-of-bounds
access or undefined behaviour in the oracle ends the run with an error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             os.path.join(ORACLE, "sanitize_check.cpp"), os.path.join(ORACLE, "ns_oracle.cpp"),
             "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "oracle sanitizer run: OK" in r.stdout
