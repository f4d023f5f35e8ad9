"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The price loop (paper_2104_00282_amd/csrc/price_loop.hpp, the host half of
the solver) runs through its CPU harness in every mode, and every entry point
of the FP64 oracle runs through a small C driver; both are built with
-fsanitize=address,undefined and stop at the first report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _compiler_supports_sanitizers(cc):
    if not shutil.which(cc):
        return False
    probe = subprocess.run([cc, *SAN, "-x", "c", "-", "-o", os.devnull], input="int main(){return 0;}",
                           capture_output=True, text=True)
    return probe.returncode == 0


@pytest.mark.skipif(not _compiler_supports_sanitizers("g++"), reason="g++ without sanitizers")
@pytest.mark.parametrize("mode", ["interior", "boundary", "subgradient", "budget", "stall",
                                  "stall_restart", "badgrad"])
def test_price_loop_under_sanitizers(tmp_path, mode):
    exe = str(tmp_path / "price_loop_san")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2104_00282_amd", "csrc"),
                           os.path.join(ROOT, "tests", "price_loop_harness.cpp"), "-o", exe])
    res = subprocess.run([exe, mode], capture_output=True, text=True, env=ENV, timeout=120)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    assert "done=1" in res.stdout


@pytest.mark.skipif(not _compiler_supports_sanitizers("gcc"), reason="gcc without sanitizers")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c99", "-fopenmp", *SAN,
                           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-o", exe,
                           "-lm"])
    env = dict(ENV, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=0")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    assert res.stdout.strip() == "ok"
