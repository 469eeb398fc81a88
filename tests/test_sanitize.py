"""The host C / C++ code under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle (``oracle/pcrit_oracle.c``) and the library's host-only preview
metric (``csrc/metrics.cpp``), built with gcc / g++ into one executable with
``tests/sanitize_driver.c``, which drives every path over small grids and bad
arguments.  Any sanitizer report ends the run with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                    reason="needs gcc and g++")
def test_host_code_sanitized(tmp_path):
    o1 = tmp_path / "oracle.o"
    o2 = tmp_path / "metrics.o"
    o3 = tmp_path / "driver.o"
    exe = tmp_path / "sanitize_driver"
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-pthread", "-c",
                           os.path.join(ROOT, "oracle", "pcrit_oracle.c"), "-o", str(o1)])
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-c",
                           os.path.join(ROOT, "paper_2009_00083_amd", "csrc", "metrics.cpp"),
                           "-o", str(o2)])
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-c",
                           os.path.join(ROOT, "tests", "sanitize_driver.c"), "-o", str(o3)])
    subprocess.check_call(["g++", *SAN, "-pthread", str(o1), str(o2), str(o3), "-o", str(exe),
                           "-lm"])
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "all checks passed" in res.stdout
