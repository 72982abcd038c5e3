"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code:
the CPU oracle (gcc) and the library's host-only translation units (the
per-size tables, the schedule table, the launch chunking; hipcc with the
sanitizers on the host side only).  Each driver under tests/sanitize/ runs
the code's entry points, error paths included, and any memory error, leak
in the oracle or undefined behaviour fails the test.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1910_06416_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, env=None, timeout=600):
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert res.returncode == 0, (" ".join(cmd)) + "\n" + res.stdout[-3000:] + res.stderr[-6000:]
    return res.stdout


@pytest.mark.slow
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "recsplit_oracle.c"),
          os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe])
    out = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert "oracle sanitizer run: ok" in out


@pytest.mark.slow
def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-pthread", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
          os.path.join(CSRC, "tables.cpp"), os.path.join(CSRC, "schedule.cpp"),
          os.path.join(HERE, "host_driver.cpp"), "-o", exe])
    # the per-size tables are cached for the life of the process on purpose
    out = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0", "HIP_VISIBLE_DEVICES": ""})
    assert "host sanitizer run: ok" in out
