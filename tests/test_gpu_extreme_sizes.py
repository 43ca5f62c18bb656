"""GPU parity at the extremes of the supported sizes.

* 256^3, the largest grid (every axis at its maximum): the Fourier solve of a
  random vector field against the FP64 oracle over the whole volume (x lines
  of 256 use the run-time x plan, 256 x 256 y-z planes the three-launch
  split solve), and the warp with its gradient at 4096 seeded voxels
  (periodic trilinear samples of the oracle at x + u(x) and at the six
  neighbours for the central differences).
* 4 x 4 x 4, the smallest: Fourier solve, ADMM iterates and a whole
  registration against the oracle.

Tolerances as in the other parity tests: Fourier solve and single iterates
1e-5 of the max norm; warp 2e-6 absolute on [0, 1] images, its central
differences 4e-6; whole registrations 1e-3 voxel and 1e-4 intensity.
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


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def f64(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_largest_grid_fourier_solve(api):
    d = (256, 256, 256)
    s = synth.random_vector_field(d, seed=90, amp=1.0)
    lam, theta, order = 0.02, 0.1, 2
    out = host(api.fourier_solve(gpu(s), lam, theta, order))
    ref = O.fourier_solve(f64(s), O.w_step_multiplier(d, lam, theta, order))
    assert np.abs(out - ref).max() < 1e-5 * np.abs(ref).max()


def test_largest_grid_warp_sampled(api):
    d = (256, 256, 256)
    nx, ny, nz = d
    img = synth.random_volume(d, seed=91, smooth_kmax=4)
    u = synth.random_vector_field(d, seed=92, amp=3.0, smooth_kmax=3)
    out, g, _ = api.warp(gpu(img), gpu(u), gpu(img), grad=True)
    out, g = host(out), host(g)
    rng = np.random.default_rng(93)
    idx = rng.choice(nx * ny * nz, size=4096, replace=False)
    z, rem = np.divmod(idx, nx * ny)
    y, x = np.divmod(rem, nx)
    I, U = f64(img), f64(u)

    def warped_at(xs, ys, zs):
        xs, ys, zs = xs % nx, ys % ny, zs % nz
        return O.sample_periodic(I, xs + U[0, zs, ys, xs], ys + U[1, zs, ys, xs], zs + U[2, zs, ys, xs])

    e = warped_at(x, y, z)
    assert np.abs(out[z, y, x] - e).max() < 2e-6
    for c, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        ej = 0.5 * (warped_at(x + dx, y + dy, z + dz) - warped_at(x - dx, y - dy, z - dz))
        assert np.abs(g[c, z, y, x] - ej).max() < 4e-6


def test_smallest_grid(api):
    d = (4, 4, 4)
    s = synth.random_vector_field(d, seed=94, amp=1.0)
    lam, theta, order = 0.2, 0.1, 2
    ref = O.fourier_solve(f64(s), O.w_step_multiplier(d, lam, theta, order))
    out = host(api.fourier_solve(gpu(s), lam, theta, order))
    assert np.abs(out - ref).max() < 1e-5 * np.abs(ref).max()

    f = synth.random_volume(d, seed=95)
    m = synth.random_volume(d, seed=96)
    _, J, r = O.warp_grad_residual(f64(m), f64(f), np.zeros((3,) + f.shape))
    J32, r32 = J.astype(np.float32), r.astype(np.float32)
    res = O.admm(f64(J32), f64(r32), lam, theta, order, 3)
    gw, gb, gv = api.admm(gpu(J32), gpu(r32), lam, theta, order, 3)
    for g_, e_ in ((gw, res.w), (gb, res.b), (gv, res.v)):
        assert np.abs(host(g_) - e_).max() < 1e-5 * np.abs(e_).max()

    reg = api.register(gpu(f), gpu(m), lam, theta, order, 3, 5)
    e = O.register(f64(f), f64(m), lam, theta, order, 3, 5)
    assert np.abs(host(reg["disp"]) - e.disp).max() < 1e-3
    assert np.abs(host(reg["warped"]) - e.warped).max() < 1e-4


def test_largest_grid_threshold_checks(api):
    """256^3 with the threshold checks running but unreachable (tolerance 0:
    no iterate repeats exactly) and switched off: both equal the fixed-count
    registration bit for bit, and every measured change is a finite
    positive number.  Three warpings, so that the warping check runs too
    (after the second warping; the last one ends the loop anyway)."""
    d = (256, 256, 256)
    f = gpu(synth.random_volume(d, seed=98, smooth_kmax=4))
    m = gpu(synth.random_volume(d, seed=99, smooth_kmax=4))
    ref = api.register(f, m, 0.01, 0.1, 2, 3, 4)
    on = api.register_threshold(f, m, 0.01, 0.1, 2, 3, 4, 0.0, 0.0)
    assert on["iters_run"] == [4, 4, 4] and on["outer_run"] == 3
    assert all(0 < x < float("inf") for c in on["admm_change"] for x in c) and len(on["admm_change"][0]) == 2
    assert len(on["warp_change"]) == 1 and 0 < on["warp_change"][0] < float("inf")
    assert torch.equal(on["disp"], ref["disp"]) and torch.equal(on["warped"], ref["warped"])
    off = api.register_threshold(f, m, 0.01, 0.1, 2, 3, 4, -1.0, -1.0)
    assert torch.equal(off["disp"], ref["disp"])
