"""The host code of the C ABI (fmnmf.cpp: validation, workspace layout,
argument checks) built with AddressSanitizer and UndefinedBehaviorSanitizer
and run on the CPU.  The kernel launchers are replaced by stubs that report
failure (tests/sanitize/stub_launch.cpp), so only the paths that return
before any device work run; tests/sanitize/host_abi_check.cpp drives them."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not found")
def test_host_abi_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_abi_check")
    srcs = [os.path.join(ROOT, "paper_1903_03237_amd", "csrc", "fmnmf.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "stub_launch.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "host_abi_check.cpp")]
    cmd = [CLANG, "-x", "c++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           *srcs, "-x", "none", "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host ABI checks passed" in r.stdout
