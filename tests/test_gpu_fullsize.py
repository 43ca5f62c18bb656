"""GPU parity at the benchmark's full size (128x128x96 heart phantom, 10 x 20),
in the launch configuration bench.py times (nadmm_register with a caller
workspace).  The whole registration is compared on a seeded sample of voxels
against stored oracle values written by tests/golden/make_golden.py; the
Fourier solve and the first ADMM iterates are compared on every voxel
against the oracle run live; the Jacobian check is compared exactly against
the oracle evaluated on the GPU's own displacement."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NAME = "phantom128x128x96"


@pytest.fixture(scope="module")
def api():
    from paper_2109_12688_amd import api as A
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A._lib.load()
    return A


@pytest.fixture(scope="module")
def pair():
    return synth.make_pair(NAME)


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", f"{NAME}_oracle_samples.json")) as f:
        return json.load(f)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def test_inputs_match_stored_oracle_run(pair, golden):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pair.fixed, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(pair.moving, dtype=np.float32).tobytes())
    assert h.hexdigest() == golden["input_sha256"], "synthetic inputs drifted: rerun make_golden.py"


def test_full_registration_sampled(api, pair, golden):
    w = synth.WORKLOADS[NAME]
    shp = pair.fixed.shape
    ws = api.workspace(shp)
    res = api.register(gpu(pair.fixed), gpu(pair.moving), w["lam"], w["theta"], w["order"],
                       w["outer"], w["iters"], ws=ws)
    idx = np.array(golden["indices"])
    disp = host(res["disp"]).reshape(3, -1)[:, idx]
    warped = host(res["warped"]).reshape(-1)[idx]
    derr = np.abs(disp - np.array(golden["disp"])).max()
    werr = np.abs(warped - np.array(golden["warped"])).max()
    print(f"full size: disp max err {derr:.3e} voxel, warped max err {werr:.3e}")
    assert derr < 1e-3
    assert werr < 1e-4
    # Jacobian: identical decisions on the same float32 field (GPU FP64 vs oracle FP64)
    stats, nneg, _ = api.jacobian(res["disp"], ws=ws)
    gd = host(res["disp"])
    mn, mx, mean, cnt = O.jacobian_stats(gd)
    s = host(stats)
    assert abs(s[0] - mn) < 1e-12 and abs(s[1] - mx) < 1e-12 and abs(s[2] - mean) < 1e-12
    assert int(nneg.cpu()[0]) == cnt
    # and close to the oracle's own registration
    gj = golden["jacobian"]
    assert abs(mn - gj["min"]) < 1e-2
    assert abs(cnt - gj["n_nonpos"]) <= gj["n_abs_below_1e-2"]


def test_full_size_fourier_solve_and_admm(api, pair):
    w = synth.WORKLOADS[NAME]
    d = w["dims"]
    s = synth.random_vector_field(d, seed=77, amp=1.0)
    ref = O.fourier_solve(s.astype(np.float64), O.w_step_multiplier(d, w["lam"], w["theta"], w["order"]))
    out = host(api.fourier_solve(gpu(s), w["lam"], w["theta"], w["order"]))
    assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-5
    # the linearised data term of the first warping, then 3 iterations
    _, J, r = O.warp_grad_residual(pair.moving.astype(np.float64), pair.fixed.astype(np.float64),
                                   np.zeros((3,) + pair.fixed.shape))
    J32, r32 = J.astype(np.float32), r.astype(np.float32)
    res = O.admm(J32.astype(np.float64), r32.astype(np.float64), w["lam"], w["theta"], w["order"], 3)
    gw, gb, gv = api.admm(gpu(J32), gpu(r32), w["lam"], w["theta"], w["order"], 3)
    for g_, e_ in ((gw, res.w), (gb, res.b), (gv, res.v)):
        assert np.abs(host(g_) - e_).max() / np.abs(e_).max() < 1e-5


# ---------------------------------------------------------------------------
# 192x192x128 phantom (n = 3, lambda = 0.005, 10 x 30), images stored as
# bfloat16 and as float32, in the launch configuration bench.py times for
# it; its y-z planes (192 x 128) exceed one workgroup's LDS, so pass B runs
# split.  This configuration's un-restarted Nesterov iteration (gamma -> 0.91
# over 30 iterations, the final map folds: min det J = -3) amplifies rounding:
# rounding the images to bfloat16 moves the FP64 oracle's own displacement
# by up to 1.26 voxel.  FP32 rounding stays within the stated bounds
# (1e-3 voxel, 1e-4 intensity) at all but a handful of the 2048 sampled
# voxels, so the bounds are asserted at 99.5 % of them, with mean errors two
# orders below the bounds and the maxima printed.
# ---------------------------------------------------------------------------
NAME4 = "phantom192x192x128"


@pytest.fixture(scope="module")
def golden4():
    with open(os.path.join(HERE, "golden", f"{NAME4}_oracle_samples.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def pair4():
    return synth.make_pair(NAME4)


@pytest.mark.parametrize("images", ["bf16", "fp32"])
def test_precision_workload_sampled(api, golden4, pair4, images):
    w = synth.WORKLOADS[NAME4]
    fb, mb = synth.bf16_bits(pair4.fixed), synth.bf16_bits(pair4.moving)
    h = hashlib.sha256()
    h.update(fb.tobytes())
    h.update(mb.tobytes())
    assert h.hexdigest() == golden4["input_sha256"], "synthetic inputs drifted: rerun make_golden.py"
    if images == "bf16":
        to_gpu = lambda b: torch.from_numpy(b.view(np.int16)).cuda().view(torch.bfloat16)  # noqa: E731
        f_img, m_img = to_gpu(fb), to_gpu(mb)
    else:
        f_img, m_img = gpu(pair4.fixed), gpu(pair4.moving)
    shp = pair4.fixed.shape
    ws = api.workspace(shp)
    res = api.register(f_img, m_img, w["lam"], w["theta"], w["order"], w["outer"], w["iters"], ws=ws)
    idx = np.array(golden4["indices"])
    disp = host(res["disp"]).reshape(3, -1)[:, idx]
    warped = host(res["warped"]).reshape(-1)[idx]
    g = golden4[images]
    derr = np.abs(disp - np.array(g["disp"])).max(axis=0)
    werr = np.abs(warped - np.array(g["warped"]))
    within = (derr <= 1e-3) & (werr <= 1e-4)
    stats, nneg, _ = api.jacobian(res["disp"], ws=ws)
    s = host(stats)
    msg = (f"{images} images: disp err max {derr.max():.3e} mean {derr.mean():.3e}; warped err max "
           f"{werr.max():.3e} mean {werr.mean():.3e}; within bounds at {within.sum()} of {len(idx)} "
           f"samples; min det J {s[0]:.4f} (oracle {g['jacobian']['min']:.4f})")
    if images == "bf16":
        f = golden4["fp32"]
        dq = np.abs(disp - np.array(f["disp"])).max(axis=0)
        msg += (f"; vs the oracle on the float32 images (storage precision): disp max "
                f"{dq.max():.3e} mean {dq.mean():.3e}")
    print(msg)
    assert within.mean() >= 0.995
    assert derr.mean() < 1e-5 and werr.mean() < 1e-6
    mn, mx, mean, cnt = O.jacobian_stats(host(res["disp"]))
    assert abs(s[0] - mn) < 1e-12 and abs(s[1] - mx) < 1e-12 and abs(s[2] - mean) < 1e-12
    assert int(nneg.cpu()[0]) == cnt
    assert abs(mn - g["jacobian"]["min"]) < 1e-2
    assert abs(cnt - g["jacobian"]["n_nonpos"]) <= g["jacobian"]["n_abs_below_1e-2"]
