"""Build libmlc.so (HIP, gfx950) in the package directory.

    python -m paper_1702_08111_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmlc.so")
SOURCES = [os.path.join(HERE, "csrc", "libmlc.hip"), os.path.join(HERE, "csrc", "server.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
    "-I", os.path.join(ROOT, "include"),
]


# The same library with its host code built with AddressSanitizer and
# UndefinedBehaviorSanitizer (device code as in libmlc.so, unsanitized);
# loaded in place of libmlc.so through MLC_LIBRARY by
# tests/test_abi_sanitized.py for the CPU-side ABI checks.
SAN_LIB = os.path.join(HERE, "libmlc_san.so")
SAN_FLAGS = [
    "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Wno-unused-result", "-Wno-unused-value",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose=True):
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(verbose=True):
    cmd = [HIPCC] + SAN_FLAGS + SOURCES + ["-o", SAN_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    return SAN_LIB


def asan_runtime():
    """The compiler's AddressSanitizer runtime (to preload into a process
    that loads SAN_LIB), or None."""
    out = subprocess.run([os.path.join(os.path.dirname(HIPCC), "amdclang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    p = out.stdout.strip()
    if p and os.path.isabs(p) and os.path.exists(p):
        return p
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


if __name__ == "__main__":
    build()
    build_sanitized()
    sys.exit(0)
