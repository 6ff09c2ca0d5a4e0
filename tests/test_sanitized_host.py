"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the host ABI tests (sizes, the host build of the constant arena at 14 and 617
buses, the error paths) run again in a subprocess against the host-sanitized
build of the library (device code unchanged), with clang's ASan runtime
preloaded.  Any report ends that process with a failure.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANGXX = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.slow


def _asan_runtime():
    if not os.path.exists(CLANGXX):
        return None
    out = subprocess.run([CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    return out if out and os.path.exists(out) else None


def test_host_code_is_clean_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    sys.path.insert(0, ROOT)
    from paper_2310_06650_amd import build
    lib = build.build(verbose=False, sanitize=True)
    env = dict(os.environ)
    env.update(QG_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail, tail
    assert "runtime error" not in tail, tail
