"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
no device code): the library's argument checks, which every form runs
before touching the device, and the CPU oracle.  Both are built with the
system C/C++ compiler into small drivers that exit non-zero on a failed
expectation; any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip("%s not available" % tool)


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r.stdout


def test_argument_checks_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "check_driver")
    _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
          "-I", os.path.join(ROOT, "paper_2602_05179_amd", "csrc"),
          os.path.join(HERE, "check_driver.cpp"),
          os.path.join(ROOT, "paper_2602_05179_amd", "csrc", "split_check.cpp"), "-o", exe], ROOT)
    assert "all expectations met" in _run([exe], ROOT)


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", *SAN, "-pthread", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "split_oracle.c"), "-lm", "-o", exe], ROOT)
    assert "all expectations met" in _run([exe], ROOT)
