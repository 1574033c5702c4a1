"""The C ABI's host validation and error paths under AddressSanitizer and
UndefinedBehaviorSanitizer: the host sources of the library (mpa_api.cpp,
ss_api.cpp) are compiled with g++ and the sanitizers, linked with a driver
(tests/host/validation_driver.cpp) that feeds them invalid parameters, maps,
batches, sizes and null handles, and run on the CPU (every call is rejected
before any device work).  The kernels' host stubs come from the built
library."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1101_0086_amd", "libmpa.so")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(LIB), reason="needs g++ and the built library")
def test_validation_paths_under_asan_and_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_1101_0086_amd", "csrc")
    srcs = [os.path.join(csrc, "mpa_api.cpp"), os.path.join(csrc, "ss_api.cpp"),
            os.path.join(ROOT, "tests", "host", "validation_driver.cpp")]
    flags = ["-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + csrc]
    objs = []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        subprocess.run(["g++"] + flags + ["-c", s, "-o", o], check=True, capture_output=True)
        objs.append(o)
    exe = str(tmp_path / "validation_driver")
    subprocess.run(["g++", "-fsanitize=address,undefined", "-o", exe] + objs +
                   [LIB, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "OK (0 failures)" in out, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]
