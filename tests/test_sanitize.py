"""The host driver under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

bse_solver.cpp and bse_smalleig.cpp are compiled with g++ against the host backend of the
kernel launchers (tests/native/host_backend.cpp, every "device" buffer a host allocation of
its exact size) and a driver program (tests/native/sanitize_main.cpp) that exercises the C ABI:
solves of every kind and precision, warm starts, the adjoint, strength scalars, Haydock and the
error paths.  Any sanitizer report, leak or failed check fails the test."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2504_10096_amd", "csrc")


def test_host_driver_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_main")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fcx-limited-range",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-w",
           os.path.join(HERE, "native", "sanitize_main.cpp"), os.path.join(HERE, "native", "host_backend.cpp"),
           os.path.join(CSRC, "bse_solver.cpp"), os.path.join(CSRC, "bse_smalleig.cpp"), "-o", exe,
           "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitizer" in r.stderr.lower() or "libasan" in r.stderr.lower():
            pytest.skip("sanitizer runtime unavailable: " + r.stderr[-300:])
        raise AssertionError(r.stderr[-3000:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-6000:])
    assert "sanitize run ok" in run.stdout
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
