"""The host half of the library (api.cpp, plan.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer by the host C++ compiler, the device launchers replaced by
stand-ins that report no device, and driven through the whole C ABI that runs without a GPU
(tests/sanitize/abi_driver.cpp). Any sanitizer report, leak included, fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_11866_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(out_dir):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    exe = os.path.join(out_dir, "abi_driver")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(HERE, "host_stubs.cpp"), os.path.join(HERE, "abi_driver.cpp"),
           "-L", os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_abi_host_paths_under_asan_ubsan(tmp_path):
    exe = _build(str(tmp_path))
    supp = tmp_path / "lsan.supp"
    # allocations the HIP runtime keeps until exit are its own, not the library's
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler-register\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=99"
    env["LSAN_OPTIONS"] = "suppressions=%s" % supp
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=98"
    env["HIP_VISIBLE_DEVICES"] = ""    # the host paths only, also where a GPU is present
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert "ERROR: LeakSanitizer" not in report, report[-4000:]
    assert "runtime error:" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert "all checks passed" in r.stdout
