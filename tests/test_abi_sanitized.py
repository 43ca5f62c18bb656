"""The host code of the library (argument validation, workspace layout,
error reporting) under AddressSanitizer and UndefinedBehaviorSanitizer: the
C-ABI checks of test_abi.py run against a build whose host code carries both
sanitizers (device code as usual), in a child process that preloads the
sanitizer runtime.  Any sanitizer report fails the child and this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_under_host_sanitizers(tmp_path):
    from paper_2109_12688_amd import build as B
    try:
        B.hipcc()
    except RuntimeError:
        pytest.skip("no ROCm toolchain")
    rt = B.asan_runtime()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("no address-sanitizer runtime for the host compiler")
    lib = B.build(out=str(tmp_path / "libnadmm_sanitized.so"), sanitize=True)
    env = dict(os.environ)
    env.update({
        "NADMM_LIBRARY": lib,
        "LD_PRELOAD": rt,
        # leaks: the interpreter and the HIP runtime keep allocations to exit
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert " passed" in res.stdout
