"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (CPU only).

- The FP64 oracle (test infrastructure): `tests/sanitizer/oracle_driver.c` compiles
  `oracle/lbm_oracle.c` into a driver that calls every entry point on small grids.
- The library's host code: `tests/sanitizer/host_driver.hip` calls the parameter
  validation, the derived constants and the host thermodynamics (`csrc/runtime_common.hpp`,
  `csrc/thermo_host.cpp`); it is built as the host pass of a HIP compile, with the
  sanitizers on that pass only, and runs no device code.

Each build aborts on the first report (-fno-sanitize-recover=all); leak checking is on.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitizer")
CSRC = os.path.join(ROOT, "paper_2112_01975_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _run(exe):
    image = open(exe, "rb").read()
    assert b"__asan_report" in image and b"__ubsan_handle" in image, "sanitizer runtime not linked"
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "ERROR: AddressSanitizer" not in report and "ERROR: LeakSanitizer" not in report
    assert "runtime error" not in report, report[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"], check=True)
    assert "oracle driver ok" in _run(exe)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_runtime_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g", "-I", CSRC,
           "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
           os.path.join(HERE, "host_driver.hip"), os.path.join(CSRC, "thermo_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    assert "host driver ok" in _run(exe)
