"""The library's host code under AddressSanitizer (CPU only).

Builds libabcs with the host half instrumented (hipcc, with -Xarch_host on
every sanitizer flag, so the GPU code is built as usual) and a C driver that
calls the host-only entry points: request sizes over a grid of descriptors,
malformed descriptors, plan creation (validation, then the host layout up to
the first device call), the launch table, the constant tables.  The build is
kept under the system temp directory, keyed by the library's source hash."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not present")
def test_host_code_under_address_sanitizer():
    from paper_2001_09632_amd import build
    key = build.build_id()
    d = os.path.join(tempfile.gettempdir(), f"abcs_asan_{key}")
    lib = os.path.join(d, "libabcs_asan.so")
    exe = os.path.join(d, "driver")
    if not os.path.exists(exe):
        os.makedirs(d, exist_ok=True)
        inc = os.path.join(ROOT, "include")
        src = os.path.join(ROOT, "paper_2001_09632_amd", "csrc", "libabcs.hip")
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                            "-I", inc, '-DABCS_BUILD_ID="asan"', "-o", lib + ".tmp", src],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        os.replace(lib + ".tmp", lib)
        r = subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address", "-fno-omit-frame-pointer", "-I", inc,
                            os.path.join(ROOT, "tests", "host_asan", "driver.c"), "-o", exe + ".tmp",
                            "-L", d, "-labcs_asan", f"-Wl,-rpath,{d}", "-lm"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        os.replace(exe + ".tmp", exe)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-3000:])
    assert r.stdout.strip().startswith("ok")
