"""The library's host code (plan building, batch layout, the server's admission and
step threads, the tuning table) under AddressSanitizer and ThreadSanitizer: a copy of
libte with instrumented host code runs the host-logic tests (dry-run server, plan
validation, workspace sizing) in a child process with the sanitizer runtime preloaded.
No GPU is used; a sanitizer report fails the child."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _runtime(kind):
    tag = {"address": "asan", "thread": "tsan"}[kind]
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.%s-x86_64.so" % tag))
    if not hits:
        pytest.skip("no %s runtime in the ROCm toolchain" % tag)
    return hits[-1]


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_code_clean_under_sanitizer(kind):
    rt = _runtime(kind)
    r = subprocess.run([sys.executable, "-m", "paper_1401_4068_amd.build", "--sanitize", kind], cwd=ROOT,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout + r.stderr
    lib = os.path.join(ROOT, "_build", kind, "libte_%s.so" % kind)
    env = dict(os.environ, TE_LIB_PATH=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=66",
               TSAN_OPTIONS="halt_on_error=1:exitcode=66:report_signal_unsafe=0")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_serve_host.py"), os.path.join("tests", "test_library_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
