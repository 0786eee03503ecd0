"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The C oracle with every entry point driven over special values and doubles
  of every magnitude (tests/sanitize/oracle_driver.c).
* The host side of libta.so (argument validation, status strings), built
  with the sanitizers on the host pass only, driven by a C program that
  passes every kind of argument the library must reject before any HIP call
  (tests/sanitize/abi_driver.c).  The GPU code of that build is the ordinary
  one; no kernel is launched.
"""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:],
                               r.stderr[-4000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-O1", "-g",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-fopenmp",
          os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "ta_oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle driver ok" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    lib = str(tmp_path / "libta_san.so")
    src = os.path.join(ROOT, "paper_2502_10831_amd", "csrc", "ta_kernels.hip")
    # sanitizers on the host pass only: each -fsanitize= follows -Xarch_host
    _run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
          "-shared", "-ffp-contract=off", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
          "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), src, "-o", lib], timeout=900)
    exe = str(tmp_path / "abi_san")
    _run([clang, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
          os.path.join(HERE, "abi_driver.c"), "-o", exe, lib,
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
          "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    r = _run([exe], env=ENV, timeout=300)
    assert "abi driver ok" in r.stdout
