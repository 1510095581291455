"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a sanitized build of the library (device code unchanged, never
run on a GPU) is loaded by tests/sanitize_driver.py with the ASan runtime
preloaded; the driver runs argument validation, NULL handling, the host
patch matrices and inverses of all 25 classes, and the complete host work of
vkmg_setup and vkmg_setup_viscosity (which stops at the first device call
without a GPU).  Any sanitizer report fails the run."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_code_is_clean_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from paper_2401_06277_amd import build as b
    try:
        lib = b.build_sanitized()
        rt = b.asan_runtime()
    except RuntimeError as e:  # no ROCm toolchain in this environment
        pytest.skip(str(e))
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_driver.py"), lib],
                         capture_output=True, text=True, env=env, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "SANITIZE-DRIVER OK" in res.stdout, out[-4000:]
    for marker in ("runtime error", "AddressSanitizer", "LeakSanitizer"):
        assert marker not in out, out[-4000:]
