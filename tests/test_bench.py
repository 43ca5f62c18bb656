"""Host logic of the benchmark (CPU): the single-GPU guard, and the committed
HBM-traffic records that the benchmark reports as `traffic` -- each must
have been taken on the kernel sources as they are (same digest) and must
read close to the algorithmic bytes of its kernel (counters far above them
would mean re-reads, far below a wrong scale)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import synth  # noqa: E402

WORKLOAD = "phantom128x128x96"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("kernel", ["pass_ca_iter", "pass_b_yz_solve"])
def test_traffic_record_matches_sources_and_bytes(kernel):
    rec = bench.stored_traffic(WORKLOAD, kernel)
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{WORKLOAD}.md")
    assert rec is not None, f"{path}: missing, or taken on other kernel sources than these"
    V = 1
    for n in synth.WORKLOADS[WORKLOAD]["dims"]:
        V *= n
    algorithmic = bench.BYTES_PER_VOXEL[kernel] * V
    assert 0.95 * algorithmic <= rec["traffic_bytes_per_launch"] <= 1.1 * algorithmic
    assert rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"] == rec["traffic_bytes_per_launch"]
    # the copy probe moved one vector field in and one out
    assert rec["copy_bytes"] == 3 * V * 4


def test_input_generation_leaves_no_process(tmp_path):
    """The benchmark's input pool (run before the GPU is touched) leaves no
    child process behind."""
    code = (
        "import sys, argparse; sys.path.insert(0, %r)\n"
        "import bench, psutil\n"
        "a = argparse.Namespace(workload='blobs32', no_bf16=True, no_grad=True, no_batch=True)\n"
        "bench.generate_inputs(a)\n"
        "print(len(psutil.Process().children(recursive=True)))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "0"
