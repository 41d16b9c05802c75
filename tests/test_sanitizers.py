"""The oracle and the host code of libswe under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

- The oracle: tests/sanitize/oracle_driver.cpp includes swe_oracle.cpp and
  runs its step, traced step, binary32 run, loss, tangent and gradient on a
  small rough state with every boundary kind, thin films and dry cells.
- The host code of the HIP library: libswe is built with the sanitizers on
  its host half only (the GPU code is unchanged), and
  tests/sanitize/abi_driver.c drives what runs without a GPU: defaults,
  validation of bad configurations, NULL handles and error messages.

Any sanitizer report fails the run (errors are not recoverable here).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return res.returncode, res.stdout + res.stderr


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-omit-frame-pointer",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                   os.path.join(HERE, "oracle_driver.cpp"), "-o", exe])
    assert rc == 0, out
    rc, out = run([exe], env=SAN_ENV, timeout=300)
    assert rc == 0 and "oracle driver: ok" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out


@pytest.mark.slow
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("the ROCm compilers are not installed")
    sys.path.insert(0, ROOT)
    from paper_1309_1230_amd import _build
    lib = str(tmp_path / "libswe_san.so")
    srcs = [os.path.join(_build.CSRC, s) for s in _build.SOURCES]
    rc, out = run([hipcc, f"--offload-arch={_build.ARCH}", "-O1", "-std=c++17", "-fPIC", "-shared",
                   "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan",
                   "-I", _build.INCLUDE, "-I", _build.CSRC, "-o", lib] + srcs)
    assert rc == 0, out
    rtdirs = [os.path.join(d, "lib", "linux")
              for d in [os.path.join("/opt/rocm/llvm/lib/clang", v)
                        for v in os.listdir("/opt/rocm/llvm/lib/clang")]]
    exe = str(tmp_path / "abi_driver")
    rc, out = run([clang, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                   "-shared-libsan", "-I", _build.INCLUDE, os.path.join(HERE, "abi_driver.c"),
                   "-L", str(tmp_path), "-lswe_san", f"-Wl,-rpath,{tmp_path}"] +
                  [f"-Wl,-rpath,{d}" for d in rtdirs] + ["-o", exe])
    assert rc == 0, out
    rc, out = run([exe], env=SAN_ENV, timeout=300)
    assert rc == 0 and "abi driver: ok" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
