"""The host-side checks of the C ABI (tests/test_abi.py) under
AddressSanitizer: the library built with its host code instrumented
(paper_2503_18056_amd.build.build_host_asan), loaded through TT_LIBRARY
into a child Python with the sanitizer's shared runtime preloaded.  No GPU:
those checks validate configurations, inputs and LDS budgets on the host."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_checks_under_asan():
    from paper_2503_18056_amd import build
    lib = build.build_host_asan()
    env = dict(os.environ, LD_PRELOAD=build.asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               TT_LIBRARY=lib)
    probe = "from paper_2503_18056_amd import _ffi; print(_ffi.load()._name)"
    r = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == lib, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_abi.py"], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stdout + r.stderr
