"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The host sources (plan runtime, coefficient generator, dispatch) are compiled with g++ and the sanitizers,
linked with a driver (tests/host_asan/driver.cpp) whose kernel entry points are stubs, and run: every
C-ABI call the driver makes returns before any HIP call (argument checks, coefficient tables for every
width, the Taylor stability bound), so no GPU is needed.  Device code is not instrumented."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_12132_amd", "csrc")
HIP_INC = "/opt/rocm/include"
HIP_LIB = "/opt/rocm/lib"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INC), reason="needs g++ and the HIP headers")
def test_host_code_under_sanitizers(tmp_path):
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I", HIP_INC, "-I", os.path.join(ROOT, "include"),
             "-I", CSRC]
    objs = []
    srcs = [os.path.join(CSRC, f) for f in ("fdetd_plan.cpp", "fdetd_coeffs.cpp", "fdetd_dispatch.cpp")]
    srcs.append(os.path.join(ROOT, "tests", "host_asan", "driver.cpp"))
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", *flags, "-c", src, "-o", obj], check=True)
        objs.append(obj)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", "-fsanitize=address,undefined", *objs, "-L", HIP_LIB, "-lamdhip64",
                    f"-Wl,-rpath,{HIP_LIB}", "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "host driver ok" in r.stdout
