"""CPU-only builds of host code under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc/g++, no GPU, no HIP):

* the FP64 oracle (oracle/oracle.c) driven through every entry point on small
  graphs with exactly sized buffers (tests/host/oracle_driver.c);
* the library's host logic (csrc/host_logic.h): the layout server's admission
  rule against a fake device and clock, parameter and CSR checks, the
  footprint bound against exact BFS counts, the cap schedules
  (tests/host/host_logic_test.cpp).

A sanitizer report or any failed check ends the program with a non-zero
status (-fno-sanitize-recover=all)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


def _needs(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} is not installed")


def test_oracle_under_sanitizers(tmp_path):
    _needs("gcc")
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", *SAN,
                    os.path.join(ROOT, "oracle", "oracle.c"),
                    os.path.join(ROOT, "tests", "host", "oracle_driver.c"), "-o", exe, "-lm"])
    assert rc == 0, out
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1")
    rc, out = _run([exe], env=env, timeout=240)
    assert rc == 0 and out.strip().startswith("OK"), out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out


def test_host_logic_under_sanitizers(tmp_path):
    _needs("g++")
    exe = str(tmp_path / "host_logic_test")
    rc, out = _run(["g++", "-std=c++17", "-Wall", *SAN,
                    os.path.join(ROOT, "tests", "host", "host_logic_test.cpp"), "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], timeout=240)
    assert rc == 0 and out.strip().startswith("OK"), out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
