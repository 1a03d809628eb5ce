"""The C ABI layer under host AddressSanitizer: api.cpp is rebuilt with the
sanitizer's instrumentation of host code only, linked with the kernels of the
normal build, and the host-side ABI tests (argument validation, status codes,
options, workspace sizes) run against it in a subprocess with the sanitizer
runtime preloaded.  Any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_under_address_sanitizer():
    from paper_2107_02736_amd import build
    if not os.path.exists(os.path.join(build.OBJDIR, "prep.hip.o")):
        pytest.skip("the library has not been built")
    try:
        runtime = build.asan_runtime()
    except RuntimeError:
        runtime = None
    if runtime is None:
        pytest.skip("no AddressSanitizer runtime next to hipcc")
    lib = build.build_asan()
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms   # the host code is instrumented
    env = dict(os.environ, LD_PRELOAD=runtime, DEANN_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert " passed" in res.stdout
