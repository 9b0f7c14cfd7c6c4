"""Host code under AddressSanitizer and UBSan (no GPU): the C-ABI layer's planning, width tables,
workspace carving and descriptor tables (spd_api.cpp built with g++ and host stand-ins for the
kernel launchers), and the FP64 oracle (oracle/planes.c), each driven over many sizes and
parameter sets.  A planted read past the oracle driver's input must be reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def run(exe):
    return subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)


def test_planner_under_asan_ubsan(tmp_path):
    need("g++")
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("ROCm headers not available")
    exe = str(tmp_path / "planner")
    src = [os.path.join(ROOT, "paper_1910_08324_amd", "csrc", "spd_api.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "launch_stubs.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "planner_driver.cpp")]
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1910_08324_amd", "csrc"),
                    "-I", "/opt/rocm/include", "-o", exe, *src, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True, capture_output=True)
    r = run(exe)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "failures 0" in r.stdout
    plans = int(r.stdout.split("plans ")[1].split(",")[0])
    assert plans > 1000


def build_oracle(tmp_path, *extra):
    exe = str(tmp_path / ("oracle" + "".join(extra).replace("-", "_")))
    subprocess.run(["gcc", *SAN, "-fopenmp", *extra, "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm"],
                   check=True, capture_output=True)
    return exe


def test_oracle_under_asan_ubsan(tmp_path):
    need("gcc")
    r = run(build_oracle(tmp_path))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "oracle driver done" in r.stdout


def test_sanitizer_reports_a_planted_overflow(tmp_path):
    need("gcc")
    r = run(build_oracle(tmp_path, "-DPLANT_OVERFLOW"))
    assert r.returncode != 0
    # UBSan's object-size check or ASan's shadow check, whichever sees it first
    assert "heap-buffer-overflow" in r.stderr or "insufficient space" in r.stderr, r.stderr
