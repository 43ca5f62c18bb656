"""GPU parity of the bfloat16-image registration (nadmm_register_bf16).

The images are stored as bfloat16 and widened exactly to float32 where they
are read, so (i) the bf16 entry point must reproduce, bit for bit, the
float32 entry point run on the same images widened to float32, and (ii) it
must meet the plain path's tolerances against the FP64 oracle run on the
bf16-rounded images (displacement 1e-3 voxel, warped intensity 1e-4).
"""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2109_12688_amd import api as A
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A._lib.load()
    return A


def bf16_pair(fixed, moving):
    f = torch.from_numpy(np.ascontiguousarray(fixed, dtype=np.float32)).cuda().to(torch.bfloat16)
    m = torch.from_numpy(np.ascontiguousarray(moving, dtype=np.float32)).cuda().to(torch.bfloat16)
    return f, m


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", ["blobs32"])
def test_bf16_equals_fp32_on_widened_images(api, name):
    w = synth.WORKLOADS[name]
    pair = synth.make_pair(name)
    fb, mb = bf16_pair(pair.fixed, pair.moving)
    a = api.register(fb, mb, w["lam"], w["theta"], w["order"], w["outer"], w["iters"],
                     return_velocities=True)
    b = api.register(fb.float().contiguous(), mb.float().contiguous(), w["lam"], w["theta"],
                     w["order"], w["outer"], w["iters"], return_velocities=True)
    assert torch.equal(a["disp"], b["disp"])
    assert torch.equal(a["warped"], b["warped"])
    assert torch.equal(a["velocities"], b["velocities"])


@pytest.mark.parametrize("d,order", [((32, 32, 32), 2), ((48, 36, 24), 3)])
def test_bf16_registration_vs_oracle(api, d, order):
    f = synth.random_volume(d, seed=21, smooth_kmax=3)
    m = synth.random_volume(d, seed=22, smooth_kmax=3)
    fb, mb = bf16_pair(f, m)
    lam, theta, outer, iters = 0.005, 0.1, 3, 8
    res = api.register(fb, mb, lam, theta, order, outer, iters)
    ref = O.register(host(fb), host(mb), lam, theta, order, outer, iters)
    assert np.abs(host(res["disp"]) - ref.disp).max() < 1e-3
    assert np.abs(host(res["warped"]) - ref.warped).max() < 1e-4


def test_bf16_rejects_mixed_dtypes(api):
    d = (16, 8, 8)
    f = torch.zeros((d[2], d[1], d[0]), device="cuda", dtype=torch.bfloat16)
    m = torch.zeros((d[2], d[1], d[0]), device="cuda", dtype=torch.float32)
    with pytest.raises(ValueError):
        api.register(f, m, 0.01, 0.1, 2, 1, 2)
