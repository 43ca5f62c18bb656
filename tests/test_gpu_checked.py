"""nadmm_register_checked through the C ABI: the registration equals
nadmm_register bit for bit, and its checks report what the oracle finds --
the divergence guard (last fixed-point residual above the first, per
warping) on a data term the un-restarted iteration cannot handle (|grad I1|
about 1, lambda = 10, n = 1) and not on the same pair with fewer iterations;
NaN in the input gives NADMM_ERR_NONFINITE; unknown flags are rejected."""
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


def _noise_pair(d, seed, amp):
    rng = np.random.default_rng(seed)
    m = (amp * rng.uniform(0, 1, size=d[::-1])).astype(np.float32)
    f = (amp * rng.uniform(0, 1, size=d[::-1])).astype(np.float32)
    return f, m


def test_checked_equals_register_when_nothing_trips(api):
    pair = synth.make_pair("blobs32")
    w = synth.WORKLOADS["blobs32"]
    f, m = torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda()
    args = (w["lam"], w["theta"], w["order"], w["outer"], w["iters"])
    ref = api.register(f, m, *args)
    res = api.register_checked(f, m, *args)
    torch.cuda.synchronize()
    assert res["status"] == 0 and res["diverged"] == [0] * w["outer"]
    assert torch.equal(res["disp"], ref["disp"]) and torch.equal(res["warped"], ref["warped"])


@pytest.mark.parametrize("iters", [60, 30])
def test_divergence_guard_matches_oracle(api, iters):
    d = (16, 12, 8)
    f, m = _noise_pair(d, 7, 3.0)
    lam, theta, order, outer = 10.0, 0.1, 1, 2
    with np.errstate(all="ignore"):
        ref = O.register(f.astype(np.float64), m.astype(np.float64), lam, theta, order, outer, iters)
    res = api.register_checked(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), lam, theta, order, outer,
                               iters)
    torch.cuda.synchronize()
    assert res["diverged"] == [int(x) for x in ref.diverged]
    finite = bool(torch.isfinite(res["disp"]).all() and torch.isfinite(res["warped"]).all())
    if not finite:
        assert res["status"] == 5
    elif any(ref.diverged):
        assert res["status"] == 6 and "diverged" in res["message"]
    else:
        assert res["status"] == 0
    assert any(ref.diverged) == (iters == 60)


def test_nonfinite_input_reported(api):
    d = (16, 12, 8)
    f, m = _noise_pair(d, 9, 1.0)
    m[3, 4, 5] = np.nan
    res = api.register_checked(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), 0.01, 0.1, 2, 2, 4,
                               divergence=False)
    assert res["status"] == 5 and "non-finite" in res["message"]
    # the guard alone does not look at values: NaN residuals count as divergence
    res = api.register_checked(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), 0.01, 0.1, 2, 2, 4,
                               finite=False)
    assert res["status"] == 6


def test_unknown_flags_rejected(api):
    import ctypes
    L = api._lib.load()
    d = (16, 12, 8)
    f = torch.zeros(d[::-1], device="cuda")
    out = torch.zeros((3,) + d[::-1], device="cuda")
    ws = api.workspace(d[::-1])
    p = api.params(0.01, 0.1, 2, 1, 3)
    st = L.nadmm_register_checked(api.dims_of(d[::-1]), ctypes.byref(p), ctypes.c_uint32(4), api._ptr(f),
                                  api._ptr(f), None, api._ptr(out), None, None, api._ptr(ws),
                                  ctypes.c_size_t(ws.numel()), api._stream())
    assert st == 1 and "flags" in L.nadmm_last_error().decode()
