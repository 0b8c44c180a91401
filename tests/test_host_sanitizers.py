"""The library's host setup code (linear-hat and order-p convolution
matrices, core matrices, the GLL rule) built with AddressSanitizer and
UndefinedBehaviorSanitizer by the host compiler (g++, no device code) and
run over meshes of several sizes, orders 1-10 and exponents 0 .. 1e6
(tests/host_sanitize/driver.cpp).  Any sanitizer report fails the test.
No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2401_04189_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC), reason="needs g++ and the HIP headers")
def test_host_setup_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_setup_san")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"), os.path.join(CSRC, "txe_fe.cpp"),
           os.path.join(CSRC, "txe_setup.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-2000:]
    # the environment is passed on unchanged apart from the sanitizer options;
    # a library preloaded into every process comes before the ASan runtime, so
    # the link-order check is relaxed
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "host setup checksum" in r.stdout, (r.stdout + r.stderr)[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
