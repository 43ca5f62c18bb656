"""Every launch shape the host code can choose, at every supported size, is
within what the kernels are compiled for (tests/launch_shape_audit.cpp:
x-line workgroups within their 768-thread launch bound, LDS budget and
per-thread item counts; y-z plane and split workgroups within theirs).
Host only: the audit includes the kernel source and runs on the CPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_launch_shape_within_kernel_bounds(tmp_path):
    from paper_2109_12688_amd import build as B
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("no ROCm toolchain")
    exe = str(tmp_path / "launch_shape_audit")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2109_12688_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "launch_shape_audit.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stdout[-4000:]
    assert " 0 violations" in run.stdout and "6188 sizes" in run.stdout, run.stdout
