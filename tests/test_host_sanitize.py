"""The library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (hipcc, sanitizers on the host side only; the
device code objects are the regular build's) and driven, from a C program,
through every entry point that runs without a GPU over valid and invalid
arguments: byte accounting, shape features, plan classes and geometry of
every (operator, direction, dtype, plan) on a grid of shapes, the register
model of every instance, the Eq. (9) model, status strings, argument checks
and handle creation.  No out-of-bounds access, no undefined operation."""
import os
import subprocess

import pytest

from paper_2609_01864_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = "-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=all".split()


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not available")
def test_host_code_under_asan_and_ubsan(lib_built, tmp_path):
    objs = [os.path.join(B.OUT_DIR, os.path.splitext(src)[0] + ".o") for src in B.SOURCES if src != "host.cpp"]
    assert all(os.path.exists(o) for o in objs), "the regular build's objects are needed"
    host = tmp_path / "host_san.o"
    cmd = [B.HIPCC, "-x", "hip", *B.FLAGS, *SAN, "-Xarch_host", "-fno-omit-frame-pointer", "-I", B.CSRC, "-c",
           os.path.join(B.CSRC, "host.cpp"), "-o", str(host)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lib = tmp_path / "libcredit_san.so"
    r = subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *SAN, "-shared-libsan", "-o", str(lib),
                        str(host), *objs], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    rt = os.path.dirname(subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                                        text=True).stdout.strip())
    exe = tmp_path / "host_sanitize"
    r = subprocess.run([CLANG, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-shared-libsan",
                        os.path.join(ROOT, "tests", "csrc", "host_sanitize_driver.c"), f"-L{tmp_path}", "-lcredit_san",
                        f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rt}", "-lm", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # leaks are not checked: the HIP runtime keeps allocations until exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert "host sanitize: ok" in run.stdout
