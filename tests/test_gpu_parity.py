"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (from the stated targets): single-step fields within 1e-5 of the
oracle relative to the field's max norm; after a whole registration, warped
intensities within 1e-4 (images in [0, 1]) and displacements within 1e-3
voxel; integer outputs (counts of non-positive Jacobians) exact.
"""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# shapes: several x-line tiles and y-z planes, odd nz, voxel counts that are
# not multiples of the 256-thread elementwise blocks (ragged tails); planes of
# 32 x 32, 64 x 48, 32 x 24 and 48 x 32 run compile-time-plan kernels, the
# others the run-time-plan kernel
SHAPES = [(8, 4, 4), (12, 6, 9), (24, 18, 9), (32, 32, 32), (48, 36, 27), (96, 64, 48), (16, 32, 24),
          (24, 48, 32)]


@pytest.fixture(scope="module")
def api():
    from paper_2109_12688_amd import api as A
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A._lib.load()
    return A


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, ref):
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-30))


def f64(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("d", SHAPES)
@pytest.mark.parametrize("amp", [0.8, 7.5])
def test_warp_gradient_residual(api, d, amp):
    img = synth.random_volume(d, seed=1, smooth_kmax=3)
    ref = synth.random_volume(d, seed=2)
    u = synth.random_vector_field(d, seed=3, amp=amp)
    out, g, r = api.warp(gpu(img), gpu(u), gpu(ref), grad=True)
    e_w = O.trilinear_periodic(f64(img), f64(u))
    assert np.abs(host(out) - e_w).max() < 2e-6
    assert np.abs(host(g) - O.gradient(f64(host(out)))).max() < 2e-6
    assert np.abs(host(r) - (host(out) - f64(ref))).max() < 1e-6
    assert np.abs(host(g) - O.gradient(e_w)).max() < 4e-6


@pytest.mark.parametrize("d", SHAPES)
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_fourier_solve(api, d, order):
    s = synth.random_vector_field(d, seed=10 + order, amp=2.0)
    lam, theta = 0.37, 0.11
    w = api.fourier_solve(gpu(s), lam, theta, order)
    ref = O.fourier_solve(f64(s), O.w_step_multiplier(d, lam, theta, order))
    assert rel(host(w), ref) < 1e-5


# y-z planes above 16384 points.  Where half a plane fits one workgroup
# (ny a multiple of 8) the x-line passes take a radix-2 step of the y
# transform and pass B transforms each half plane in one workgroup (the first
# three); otherwise pass B runs as three launches (rows, columns, rows; the
# last: ny = 162)
SPLIT_SHAPES = [(8, 144, 128), (12, 192, 96), (16, 96, 192), (8, 162, 108)]


@pytest.mark.parametrize("d", SPLIT_SHAPES)
@pytest.mark.parametrize("order", [1, 3])
def test_fourier_solve_split_planes(api, d, order):
    s = synth.random_vector_field(d, seed=40 + order, amp=2.0)
    lam, theta = 0.21, 0.13
    w = api.fourier_solve(gpu(s), lam, theta, order)
    ref = O.fourier_solve(f64(s), O.w_step_multiplier(d, lam, theta, order))
    assert rel(host(w), ref) < 1e-5


def test_admm_split_planes(api):
    d = (12, 192, 96)
    f = synth.random_volume(d, seed=44, smooth_kmax=3)
    m = synth.random_volume(d, seed=45, smooth_kmax=3)
    _, J, r = O.warp_grad_residual(f64(m), f64(f), np.zeros((3,) + f.shape))
    J32, r32 = J.astype(np.float32), r.astype(np.float32)
    res = O.admm(f64(J32), f64(r32), 0.005, 0.1, 3, 4)
    gw, gb, gv = api.admm(gpu(J32), gpu(r32), 0.005, 0.1, 3, 4)
    for g_, e_ in ((gw, res.w), (gb, res.b), (gv, res.v)):
        assert rel(host(g_), e_) < 2e-5


def test_fourier_solve_plane_wave_and_dc(api):
    d = (32, 24, 18)
    nx, ny, nz = d
    xx, yy, zz = synth.grid(d)
    lam, theta, order = 0.5, 0.1, 2
    m = O.w_step_multiplier(d, lam, theta, order, half=False)
    for (p, q, r) in [(0, 0, 0), (1, 0, 0), (nx // 2, 3, 2), (5, ny // 2, nz // 2), (0, 7, 4), (nx // 2, 0, 1)]:
        wave = np.cos(2 * np.pi * (p * xx / nx + q * yy / ny + r * zz / nz))
        out = host(api.fourier_solve(gpu(np.stack([wave] * 3)), lam, theta, order))
        assert np.abs(out[1] - m[r, q, p] * wave).max() < 2e-6


def _jr(d, seed, jscale=0.3):
    rng = np.random.default_rng(seed)
    nx, ny, nz = d
    J = (jscale * rng.standard_normal((3, nz, ny, nx))).astype(np.float32)
    r = (0.3 * rng.standard_normal((nz, ny, nx))).astype(np.float32)
    return J, r


@pytest.mark.parametrize("d", [(8, 4, 4), (24, 18, 9), (32, 32, 32), (96, 64, 48)])
@pytest.mark.parametrize("iters", [1, 2, 3, 10])
@pytest.mark.parametrize("data_term", [2, 1])
def test_admm_iterates(api, d, iters, data_term):
    J, r = _jr(d, 20 + iters)
    lam, theta, order = 0.05, 0.1, 2
    w, b, v = api.admm(gpu(J), gpu(r), lam, theta, order, iters, data_term=data_term, eps=1e-8)
    ref = O.admm(f64(J), f64(r), lam, theta, order, iters, data_term=data_term, eps=1e-8)
    tol = 1e-5 if iters <= 3 else 5e-5
    assert rel(host(w), ref.w) < tol
    assert rel(host(b), ref.b) < tol
    assert rel(host(v), ref.v) < tol


@pytest.mark.parametrize("d", [(12, 6, 9), (32, 32, 32), (48, 36, 27)])
def test_compose_and_expmap(api, d):
    u = synth.random_vector_field(d, seed=30, amp=3.0, smooth_kmax=3)
    v = synth.random_vector_field(d, seed=31, amp=2.0, smooth_kmax=3)
    c = api.compose(gpu(u), gpu(v))
    assert np.abs(host(c) - O.compose(f64(u), f64(v))).max() < 1e-5
    for steps in (0, 1, 6):
        e = api.expmap(gpu(v), steps)
        assert np.abs(host(e) - O.expmap(f64(v), steps)).max() < 2e-5


@pytest.mark.parametrize("d", [(12, 6, 9), (32, 32, 32), (96, 64, 48)])
def test_jacobian(api, d):
    # amplitude grows with the grid so that folds (det <= 0) occur at every size
    u = synth.random_vector_field(d, seed=40, amp=max(2.5, 0.12 * d[0]), smooth_kmax=4)
    stats, nneg, det = api.jacobian(gpu(u), want_det=True)
    ed = O.jacobian_det(f64(u))
    mn, mx, mean, cnt = O.jacobian_stats(f64(u))
    s = host(stats)
    assert abs(s[0] - mn) < 1e-12 and abs(s[1] - mx) < 1e-12 and abs(s[2] - mean) < 1e-12
    assert int(nneg.cpu()[0]) == cnt
    assert np.abs(host(det) - ed).max() < 1e-6 * max(1.0, np.abs(ed).max())
    assert cnt > 0  # the amplitude is chosen so folds occur: the count is exercised


def test_identity_registration_is_exactly_zero(api):
    img = synth.random_volume((32, 24, 18), seed=5, smooth_kmax=3)
    res = api.register(gpu(img), gpu(img), 0.01, 0.1, 2, 3, 5, return_velocities=True)
    assert torch.count_nonzero(res["disp"]).item() == 0
    assert torch.count_nonzero(res["velocities"]).item() == 0
    assert torch.equal(res["warped"], gpu(img))


def test_register_blobs32(api):
    w = synth.WORKLOADS["blobs32"]
    pair = synth.make_pair("blobs32")
    res = api.register(gpu(pair.fixed), gpu(pair.moving), w["lam"], w["theta"], w["order"],
                       w["outer"], w["iters"], return_velocities=True)
    ref = O.register(f64(pair.fixed), f64(pair.moving), w["lam"], w["theta"], w["order"],
                     w["outer"], w["iters"], keep_velocities=True)
    assert np.abs(host(res["disp"]) - ref.disp).max() < 1e-3
    assert np.abs(host(res["warped"]) - ref.warped).max() < 1e-4
    vel = host(res["velocities"])
    for c in range(w["outer"]):
        assert rel(vel[c], ref.velocities[c]) < 1e-3
    stats, nneg, _ = api.jacobian(res["disp"])
    mn, _, _, cnt = O.jacobian_stats(ref.disp)
    assert int(nneg.cpu()[0]) == cnt == 0
    assert abs(host(stats)[0] - mn) < 1e-3


def test_register_init_disp_and_outer0(api):
    d = (24, 18, 12)
    f = synth.random_volume(d, seed=6, smooth_kmax=3)
    m = synth.random_volume(d, seed=7, smooth_kmax=3)
    u0 = synth.random_vector_field(d, seed=8, amp=1.0, smooth_kmax=2)
    res = api.register(gpu(f), gpu(m), 0.02, 0.1, 1, 2, 4, init_disp=gpu(u0))
    ref = O.register(f64(f), f64(m), 0.02, 0.1, 1, 2, 4, init_disp=f64(u0))
    assert np.abs(host(res["disp"]) - ref.disp).max() < 1e-4
    z = api.register(gpu(f), gpu(m), 0.02, 0.1, 1, 0, 4, init_disp=gpu(u0))
    assert np.array_equal(host(z["disp"]), f64(u0))
    assert np.abs(host(z["warped"]) - O.trilinear_periodic(f64(m), f64(u0))).max() < 2e-6


def test_register_l1_data_term(api):
    w = synth.WORKLOADS["blobs32"]
    pair = synth.make_pair("blobs32")
    res = api.register(gpu(pair.fixed), gpu(pair.moving), 0.05, 0.1, 3, 3, 10, data_term=1, eps=1e-8)
    ref = O.register(f64(pair.fixed), f64(pair.moving), 0.05, 0.1, 3, 3, 10, data_term=1)
    assert np.abs(host(res["disp"]) - ref.disp).max() < 1e-3


def test_determinism(api):
    pair = synth.make_pair("blobs32")
    a = api.register(gpu(pair.fixed), gpu(pair.moving), 0.01, 0.1, 2, 2, 6)
    b = api.register(gpu(pair.fixed), gpu(pair.moving), 0.01, 0.1, 2, 2, 6)
    assert torch.equal(a["disp"], b["disp"]) and torch.equal(a["warped"], b["warped"])


def test_pyramid_vs_oracle(api):
    """Three levels (16x16x12, 32x32x24, 64x64x48) with the paper's caps of
    its first hyper-parameter version: warpings 10, 10, 5 and iterations
    10, 5, 5."""
    d = (64, 64, 48)
    f = synth.random_volume(d, seed=130, smooth_kmax=3)
    m = synth.random_volume(d, seed=131, smooth_kmax=3)
    res = api.register_pyramid(gpu(f), gpu(m), 0.01, 0.1, 2)
    ref = O.pyramid_register(f64(f), f64(m), 0.01, 0.1, 2, outer=(10, 10, 5), iters=(10, 5, 5))
    assert np.abs(host(res["disp"]) - ref.disp).max() < 1e-3
    assert np.abs(host(res["warped"]) - ref.warped).max() < 1e-4
    # one level is a plain registration
    one = api.register_pyramid(gpu(f), gpu(m), 0.01, 0.1, 2, outer=(2,), iters=(3,))
    plain = api.register(gpu(f), gpu(m), 0.01, 0.1, 2, 2, 3)
    assert torch.equal(one["disp"], plain["disp"])


def test_count_nonfinite(api):
    """Exact count of NaN / +-inf entries (integer result, so exact equality):
    none, a few at known positions (first, last, across components), and 1000
    seeded positions in a field large enough for the grid-stride loop."""
    d = (24, 18, 9)
    u = synth.random_vector_field(d, seed=50, amp=1.0)
    assert api.count_nonfinite(gpu(u)).item() == 0
    flat = u.reshape(-1).copy()
    bad = [0, 7, flat.size // 2, flat.size - 1]
    for i, v in zip(bad, (np.nan, np.inf, -np.inf, np.nan)):
        flat[i] = v
    u2 = flat.reshape(u.shape)
    assert api.count_nonfinite(gpu(u2)).item() == 4
    assert [api.count_nonfinite(gpu(u2[c])).item() for c in range(3)] == [2, 1, 1]
    big = synth.random_vector_field((128, 128, 96), seed=51, amp=1.0).reshape(-1)
    pos = np.random.default_rng(52).choice(big.size, size=1000, replace=False)
    big[pos] = np.nan
    assert api.count_nonfinite(gpu(big.reshape((3, 96, 128, 128)))).item() == 1000
