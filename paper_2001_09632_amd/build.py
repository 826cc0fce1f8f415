"""Build libabcs.so (gfx950 HIP kernels + C ABI) in place with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libabcs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in VGPRs (no AGPR round trip before each use)
    "-mllvm", "--amdgpu-mfma-vgpr-form",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)) + [
        os.path.join(os.path.dirname(PKG), "include", "abcs.h")]


def build_id():
    """SHA-256 (first 16 hex digits) of the sources and the compiler flags:
    the library reports it (abcs_build_id), and launch-tuning results are
    kept under it."""
    import hashlib
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for f in sources():
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def build(verbose=False):
    """Compile libabcs.so; raises CalledProcessError on failure."""
    inc = os.path.join(os.path.dirname(PKG), "include")
    cmd = [HIPCC] + FLAGS + ["-I", inc, f'-DABCS_BUILD_ID="{build_id()}"', "-o", LIB + ".tmp",
                             os.path.join(CSRC, "libabcs.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise subprocess.CalledProcessError(res.returncode, cmd)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
