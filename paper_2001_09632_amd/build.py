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


def code_text(data):
    """C / C++ source bytes without their comments, trailing blanks and empty
    lines: what the compiler sees apart from line numbers, so that edits of
    comments alone keep a build's id (and the launch tuning stored under it)."""
    out = bytearray()
    i, n = 0, len(data)
    while i < n:
        c = data[i:i + 1]
        if c in (b'"', b"'"):                       # string or character literal, kept whole
            j = i + 1
            while j < n and data[j:j + 1] != c:
                j += 2 if data[j:j + 1] == b"\\" else 1
            out += data[i:j + 1]
            i = j + 1
        elif data.startswith(b"//", i):
            while i < n and data[i:i + 1] != b"\n":
                i += 1
        elif data.startswith(b"/*", i):
            j = data.find(b"*/", i + 2)
            i = n if j < 0 else j + 2
            out += b" "
        else:
            out += c
            i += 1
    lines = (ln.rstrip() for ln in bytes(out).split(b"\n"))
    return b"\n".join(ln for ln in lines if ln)


def build_id():
    """SHA-256 (first 16 hex digits) of the sources' code (code_text) and the
    compiler flags: the library reports it (abcs_build_id), and launch-tuning
    results are kept under it."""
    import hashlib
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for f in sources():
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + code_text(fh.read()))
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
