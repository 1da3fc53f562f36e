"""The CPU-side ABI checks (tests/test_abi_cpu.py) again, in a child process
that loads the host-sanitized build of the library (libmlc_san.so: host code
with AddressSanitizer and UndefinedBehaviorSanitizer, no device code) with
the sanitizer runtime preloaded: problem validation, sizing, autotune bounds,
status strings and the error paths of the context, plan and server calls run
with every host memory access and arithmetic operation checked."""
import os
import subprocess
import sys

import pytest

from paper_1702_08111_amd import build as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_under_sanitizers():
    if not os.path.exists(b.SAN_LIB):
        pytest.skip("libmlc_san.so is not built (__graft_entry__.build() builds it)")
    rt = b.asan_runtime()
    assert rt, "the compiler's AddressSanitizer runtime was not found"
    env = dict(os.environ)
    env["MLC_LIBRARY"] = b.SAN_LIB
    # the runtime first, anything already preloaded after it
    env["LD_PRELOAD"] = rt + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    # the child really maps the sanitizer runtime and the sanitized library
    probe = ("from paper_1702_08111_amd import mlc; mlc.lib(); m = open('/proc/self/maps').read(); "
             "print('libclang_rt.asan' in m, 'libmlc_san.so' in m)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.split() == ["True", "True"], (r.stdout, r.stderr[-2000:])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
