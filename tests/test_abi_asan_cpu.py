"""The ABI's host-side argument checks under AddressSanitizer: tests/test_abi_cpu.py run
against a build of the library whose host code is instrumented (the sanitizer runtime
preloaded into the test process). No GPU is used; the build is reused while it is newer
than the library's sources."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib):
    if not os.path.exists(lib):
        return True
    srcs = glob.glob(os.path.join(ROOT, "paper_1003_0524_amd", "csrc", "*")) + \
        glob.glob(os.path.join(ROOT, "include", "*.h"))
    return os.path.getmtime(lib) < max(os.path.getmtime(s) for s in srcs)


def test_abi_checks_run_clean_under_address_sanitizer():
    from paper_1003_0524_amd import build
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    lib = build.ASAN_LIB
    if _stale(lib):
        build.build_asan(lib)
    env = dict(os.environ, EXC_LIBRARY=lib, LD_PRELOAD=build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0 and " passed" in out, out[-4000:]
    # the library in use was the instrumented one
    nm = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in nm
