"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, g++ / gcc).

The library's host parts (angle sets, segment tables, sweep plans, the tuning cache) and the oracle are
built with -fsanitize=address,undefined into small drivers (tests/sanitize/) and run; any report fails
the test.  Device code is not built here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, cwd, env=None):
    res = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    return res.stdout


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_and_oracle_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1107_5719_amd", "csrc")
    host = str(tmp_path / "host_driver")
    _run(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
          os.path.join(csrc, "geometry.cpp"), os.path.join(csrc, "tune_cache.cpp"), "-o", host], ROOT)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = _run([host, str(tmp_path / "cache.json")], ROOT, env)
    assert "host driver ok" in out
    orc = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=gnu11", "-fopenmp", *SAN, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", orc], ROOT)
    out = _run([orc], ROOT, env)
    assert "oracle driver ok" in out
