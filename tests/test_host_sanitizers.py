"""The library's host C++ table generator under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host/table_driver.cpp drives table creation (Levenberg-Marquardt, Cholesky, Householder QR), export,
the exact kernel, the correction and the map error through the C ABI; it is compiled together with
csrc/table.cpp by g++ with -fsanitize=address,undefined (host code only: the file's only HIP call is a
copy that the driver reaches with a NULL buffer, which returns before it). Any sanitizer report fails."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_07102_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"), reason="no g++ / ROCm")
def test_table_generator_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "table_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "table_driver.cpp"),
           os.path.join(CSRC, "table.cpp"), "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "table driver: ok" in r.stdout
