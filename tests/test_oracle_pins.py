"""Pins for the FP64 oracle: each test checks it against something the paper or
the mathematics fixes, never against a re-typed copy of its own formula.

Dense reference operators below are assembled from the stencils with explicit
index loops (not the oracle's roll-based differences), on grids small enough
for dense linear algebra.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
import synth


# ---------------------------------------------------------------------------
# dense reference operators (explicit index loops on tiny grids)
# ---------------------------------------------------------------------------
def _idx(x, y, z, d):
    nx, ny, nz = d
    return x + nx * (y + ny * z)


def dense_neg_laplacian(d):
    """The periodic 7-point -Delta with unit spacing as a V x V matrix."""
    nx, ny, nz = d
    V = nx * ny * nz
    L = np.zeros((V, V))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = _idx(x, y, z, d)
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    L[i, i] += 1.0
                    L[i, _idx((x + dx) % nx, (y + dy) % ny, (z + dz) % nz, d)] -= 1.0
    return L


def dense_central_diff(d, axis_xyz):
    nx, ny, nz = d
    V = nx * ny * nz
    D = np.zeros((V, V))
    step = [(1, 0, 0), (0, 1, 0), (0, 0, 1)][axis_xyz]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = _idx(x, y, z, d)
                jp = _idx((x + step[0]) % nx, (y + step[1]) % ny, (z + step[2]) % nz, d)
                jm = _idx((x - step[0]) % nx, (y - step[1]) % ny, (z - step[2]) % nz, d)
                D[i, jp] += 0.5
                D[i, jm] -= 0.5
    return D


def flat(f):
    """(nz, ny, nx) -> x-fastest vector, matching _idx."""
    return f.reshape(-1)


def model_minimiser(J, r, lam, order):
    """Brute-force minimiser of Eq. (2) with s = 2 for the regulariser
    <v, (-Delta_h)^n v>: solve (blockdiag(J J^T) + lam I_3 (x) L^n) v = -J r."""
    d = (J.shape[3], J.shape[2], J.shape[1])
    V = J[0].size
    Ln = np.linalg.matrix_power(dense_neg_laplacian(d), order)
    Jf = J.reshape(3, V)
    A = np.zeros((3 * V, 3 * V))
    for c in range(3):
        for e in range(3):
            A[c * V + np.arange(V), e * V + np.arange(V)] += Jf[c] * Jf[e]
        A[c * V:(c + 1) * V, c * V:(c + 1) * V] += lam * Ln
    rhs = -(Jf * r.reshape(V)).reshape(-1)
    return np.linalg.solve(A, rhs).reshape(J.shape)


# ---------------------------------------------------------------------------
# P1  Nesterov scalars (Sec. 3, Eq. (5))
# ---------------------------------------------------------------------------
def test_p1_nesterov_scalars():
    a = O.nesterov_alphas(40)
    g = O.nesterov_gammas(40)
    assert a[0] == 1.0
    # alpha^1 is the golden ratio; gamma_0 = 0 exactly (no momentum at k = 0, 1)
    assert a[1] == pytest.approx((1 + math.sqrt(5)) / 2, abs=1e-15)
    assert g[0] == 0.0
    # every alpha^{k+1} is the positive root of t^2 - t - (alpha^k)^2 = 0
    for k in range(40):
        t = a[k + 1]
        assert t * t - t == pytest.approx(a[k] ** 2, rel=1e-14)
        assert t > 0
    # growth bounds of the accelerated sequence: (k+2)/2 <= alpha^k <= k+1
    for k in range(1, 41):
        assert (k + 2) / 2.0 <= a[k] <= k + 1
    # gamma_1 from the closed form of alpha^1, alpha^2
    phi = (1 + math.sqrt(5)) / 2
    assert g[1] == pytest.approx((phi - 1) / ((1 + math.sqrt(1 + 4 * phi * phi)) / 2), rel=1e-15)
    assert np.all(np.diff(g) > 0) and g[-1] < 1.0


# The first extrapolation weights of Eq. (5), gamma_k = (alpha^k - 1) / alpha^{k+1}
# with alpha^0 = 1, typed in to ten digits (evaluated once from the printed
# recurrence, independently of the oracle).
TYPED_GAMMAS = (0.0, 0.2817535251, 0.4340427828, 0.5310638054)


def dense_admm_schedule(J, r, lam, theta, order, gammas):
    """Eq. (5) written out with dense operators on a tiny grid, iteration by
    iteration in the paper's order, with the extrapolation weight of each step
    taken from ``gammas``: iteration k uses w_hat^k = w^{k-1} +
    gammas[k-1] (w^{k-1} - w^{k-2}) (likewise b_hat), w^{-1} = b^{-1} = 0 and
    w_hat^0 = b_hat^0 = 0.  The v-step is a dense 3x3 solve per voxel, the
    w-step a dense solve of (lambda L^n + theta I) w = theta (v + b_hat)."""
    d = (J.shape[3], J.shape[2], J.shape[1])
    V = J[0].size
    A = lam * np.linalg.matrix_power(dense_neg_laplacian(d), order) + theta * np.eye(V)
    Jf = J.reshape(3, V)
    rf = r.reshape(V)
    zero = np.zeros((3, V))
    w_hat, b_hat, w_prev, b_prev = zero, zero, zero, zero
    out = []
    for k in range(len(gammas) + 1):
        a = w_hat - b_hat
        v = np.empty((3, V))
        for i in range(V):
            M = np.outer(Jf[:, i], Jf[:, i]) + theta * np.eye(3)
            v[:, i] = np.linalg.solve(M, theta * a[:, i] - Jf[:, i] * rf[i])
        w = np.stack([np.linalg.solve(A, theta * (v[c] + b_hat[c])) for c in range(3)])
        b = b_hat + v - w
        out.append((v.reshape(J.shape), w.reshape(J.shape), b.reshape(J.shape)))
        if k < len(gammas):
            g = gammas[k]
            w_hat = w + g * (w - w_prev)
            b_hat = b + g * (b - b_prev)
            w_prev, b_prev = w, b
    return out


def test_p1b_extrapolation_schedule_against_dense_recurrence():
    """Iterates v^k, w^k, b^k for k = 0..4 of the oracle's ADMM equal the dense
    evaluation of Eq. (5) with the typed-in gamma_0..gamma_3 (gamma_1 first
    enters at iteration 2).  The same dense recurrence with the weights
    shifted by one index (iteration k extrapolating with gamma_k) is a
    different trajectory, so an index mistake in the oracle fails here."""
    rng = np.random.default_rng(22)
    J = rng.uniform(0.1, 0.4, size=(3, 4, 4, 4)) * rng.choice([-1, 1], size=(3, 4, 4, 4))
    r = rng.uniform(-0.5, 0.5, size=(4, 4, 4))
    lam, theta, order = 0.5, 0.1, 2
    res = O.admm(J, r, lam, theta, order, 5, history=True)
    assert np.allclose(res.gammas[:4], TYPED_GAMMAS, rtol=0, atol=1e-10)
    ref = dense_admm_schedule(J, r, lam, theta, order, TYPED_GAMMAS)
    for k, (v, w, b) in enumerate(ref):
        h = res.history[k]
        for name, got, want in (("v", h["v"], v), ("w", h["w"], w), ("b", h["b"], b)):
            err = np.abs(got - want).max() / np.abs(want).max()
            assert err < 1e-9, (k, name, err)
    # discriminating power: the schedule shifted by one index (gamma_k at
    # iteration k) already differs at iteration 1, and by far more than the
    # tolerance above from iteration 2 on
    shifted = dense_admm_schedule(J, r, lam, theta, order, TYPED_GAMMAS[1:] + (0.5987785941,))
    for k in (1, 2, 3, 4):
        err = np.abs(shifted[k][1] - ref[k][1]).max() / np.abs(ref[k][1]).max()
        assert err > 1e-3, (k, err)
    # and so does the schedule without momentum (every gamma zero)
    plain = dense_admm_schedule(J, r, lam, theta, order, (0.0, 0.0, 0.0, 0.0))
    assert np.abs(plain[1][1] - ref[1][1]).max() == 0.0  # gamma_0 = 0: iterations 0, 1 agree
    for k in (2, 3, 4):
        assert np.abs(plain[k][1] - ref[k][1]).max() / np.abs(ref[k][1]).max() > 1e-3, k


# ---------------------------------------------------------------------------
# P2  Laplacian symbol (Sec. 3, text after Eq. (6))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [(4, 4, 4), (5, 5, 5), (6, 4, 3)])
def test_p2_symbol_is_dense_laplacian_spectrum(d):
    L = dense_neg_laplacian(d)
    sym = O.laplacian_symbol(d, half=False)
    # sorted spectrum equals the symbol over the full DFT grid
    ev = np.linalg.eigvalsh(L)
    assert np.allclose(np.sort(ev), np.sort(sym.ravel()), atol=1e-12)
    # every plane wave is an eigenvector with the symbol as eigenvalue
    nx, ny, nz = d
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for (p, q, r) in [(1, 0, 0), (0, 1, 2), (2, 3, 1), (nx - 1, ny - 1, nz - 1)]:
        e = np.exp(2j * np.pi * (p * xx / nx + q * yy / ny + r * zz / nz))
        Le = L @ flat(e)
        assert np.allclose(Le, sym[r, q, p] * flat(e), atol=1e-12)
    assert sym[0, 0, 0] == 0.0 and np.all(sym >= 0)


# ---------------------------------------------------------------------------
# P3  Sherman-Morrison v-step (Eq. (6), s = 2)
# ---------------------------------------------------------------------------
def test_p3_sherman_morrison_matches_dense_3x3():
    rng = np.random.default_rng(3)
    d = (5, 4, 3)
    J = rng.standard_normal((3, 3, 4, 5))
    a = rng.standard_normal((3, 3, 4, 5))
    r = rng.standard_normal((3, 4, 5))
    theta = 0.37
    v = O.v_step_l2(a, J, r, theta)
    for z in range(3):
        for y in range(4):
            for x in range(5):
                j = J[:, z, y, x]
                M = np.outer(j, j) + theta * np.eye(3)
                ref = np.linalg.solve(M, theta * a[:, z, y, x] - j * r[z, y, x])
                assert np.allclose(v[:, z, y, x], ref, rtol=1e-13, atol=1e-14)
    # v minimises the data subproblem: gradient vanishes
    rho = np.sum(J * v, axis=0) + r
    grad = J * rho[None] + theta * (v - a)
    assert np.abs(grad).max() < 1e-12


def test_p3b_l1_vstep_minimises_subproblem():
    """s = 1: v minimises |<J,v> + r| + theta/2 |v - a|^2 per voxel (checked
    by a 1-D search along J, the only direction the data term sees)."""
    rng = np.random.default_rng(4)
    J = rng.standard_normal((3, 2, 2, 2))
    a = rng.standard_normal((3, 2, 2, 2))
    r = rng.standard_normal((2, 2, 2))
    theta = 0.5
    v = O.v_step_l1(a, J, r, theta, eps=0.0)
    for idx in np.ndindex(2, 2, 2):
        j, aa, rr, vv = J[(slice(None),) + idx], a[(slice(None),) + idx], r[idx], v[(slice(None),) + idx]
        f = lambda u: abs(j @ u + rr) + theta / 2 * np.sum((u - aa) ** 2)
        ts = np.linspace(-5, 5, 200001)
        best = min(f(aa + t * j) for t in ts[::50])
        assert f(vv) <= best + 1e-6


# ---------------------------------------------------------------------------
# P4  Fourier w-step (Eq. (6) bottom, read with theta in the numerator)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,order", [((4, 4, 4), 1), ((4, 4, 4), 2), ((6, 4, 3), 3), ((5, 3, 4), 2)])
def test_p4_fourier_solve_equals_dense_solve(d, order):
    rng = np.random.default_rng(11)
    lam, theta = 0.7, 0.2
    nx, ny, nz = d
    s = rng.standard_normal((3, nz, ny, nx))
    w = O.fourier_solve(s, O.w_step_multiplier(d, lam, theta, order))
    A = lam * np.linalg.matrix_power(dense_neg_laplacian(d), order) + theta * np.eye(nx * ny * nz)
    for c in range(3):
        ref = np.linalg.solve(A, theta * flat(s[c]))
        assert np.allclose(flat(w[c]), ref, rtol=1e-12, atol=1e-13)


def test_p4_plane_wave_dc_and_self_adjoint():
    d = (8, 6, 4)
    nx, ny, nz = d
    lam, theta, order = 0.3, 0.1, 2
    m = O.w_step_multiplier(d, lam, theta, order)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p, q, r = 3, 2, 1
    wave = np.cos(2 * np.pi * (p * xx / nx + q * yy / ny + r * zz / nz))
    k = (2 * (3 - np.cos(2 * np.pi * p / nx) - np.cos(2 * np.pi * q / ny) - np.cos(2 * np.pi * r / nz))) ** order
    out = O.fourier_solve(np.stack([wave] * 3), m)
    assert np.allclose(out[0], theta / (theta + lam * k) * wave, atol=1e-14)
    const = np.full((3, nz, ny, nx), 2.5)
    assert np.allclose(O.fourier_solve(const, m), const, atol=1e-14)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, 3, nz, ny, nx))
    assert np.sum(O.fourier_solve(x, m) * y) == pytest.approx(np.sum(x * O.fourier_solve(y, m)), rel=1e-12)


# ---------------------------------------------------------------------------
# P5  whole ADMM against the brute-force minimiser of the model (4^3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order,lam", [(1, 0.1), (2, 0.01), (2, 0.5), (3, 0.1)])
def test_p5_admm_converges_to_dense_minimiser(order, lam):
    rng = np.random.default_rng(100 + order)
    J = rng.uniform(-0.3, 0.3, size=(3, 4, 4, 4))
    r = rng.uniform(-0.5, 0.5, size=(4, 4, 4))
    vstar = model_minimiser(J, r, lam, order)
    res = O.admm(J, r, lam, 0.1, order, 1000)
    scale = np.abs(vstar).max()
    assert np.abs(res.w - vstar).max() / scale < 1e-10
    assert np.abs(res.v - vstar).max() / scale < 1e-10


def test_p5_planted_literal_wstep_fails():
    """The w-step as printed (no theta in the numerator) does not reach the
    model's minimiser: the pins above reject that reading."""
    rng = np.random.default_rng(102)
    d = (4, 4, 4)
    J = rng.uniform(-0.3, 0.3, size=(3, 4, 4, 4))
    r = rng.uniform(-0.5, 0.5, size=(4, 4, 4))
    lam, theta, order = 0.01, 0.1, 2
    vstar = model_minimiser(J, r, lam, order)
    literal = 1.0 / (lam * O.laplacian_symbol(d) ** order + theta)
    with np.errstate(all="ignore"):
        res = O.admm(J, r, lam, theta, order, 300, mult=literal)
        err = np.abs(res.w - vstar).max() / np.abs(vstar).max()
    assert not (err < 1e-3)


# ---------------------------------------------------------------------------
# P6  special cases
# ---------------------------------------------------------------------------
def test_p6_lambda_zero_gives_normal_flow():
    rng = np.random.default_rng(6)
    J = rng.uniform(0.2, 0.6, size=(3, 4, 4, 4)) * rng.choice([-1, 1], size=(3, 4, 4, 4))
    r = rng.uniform(-0.5, 0.5, size=(4, 4, 4))
    res = O.admm(J, r, 0.0, 0.1, 2, 400)
    normal = -J * (r / np.sum(J * J, axis=0))[None]
    assert np.abs(res.w - normal).max() < 1e-10


def test_p6_first_iteration_from_zero():
    rng = np.random.default_rng(7)
    d = (6, 4, 4)
    J = rng.standard_normal((3, 4, 4, 6))
    r = rng.standard_normal((4, 4, 6))
    lam, theta, order = 0.2, 0.3, 1
    res = O.admm(J, r, lam, theta, order, 1)
    v0 = -J * (r / (theta + np.sum(J * J, axis=0)))[None]
    A = lam * dense_neg_laplacian(d) + theta * np.eye(96)
    w0 = np.stack([np.linalg.solve(A, theta * flat(v0[c])).reshape(4, 4, 6) for c in range(3)])
    assert np.allclose(res.v, v0, atol=1e-14)
    assert np.allclose(res.w, w0, atol=1e-13)
    assert np.allclose(res.b, v0 - w0, atol=1e-13)


# ---------------------------------------------------------------------------
# P7  identity: fixed == moving gives exactly zero
# ---------------------------------------------------------------------------
def test_p7_identity_is_exact_zero():
    img = synth.random_volume((12, 10, 8), seed=3, smooth_kmax=3).astype(np.float64)
    res = O.register(img, img, 0.01, 0.1, 2, 3, 5)
    assert np.count_nonzero(res.disp) == 0
    assert np.array_equal(res.warped, img)


# ---------------------------------------------------------------------------
# P8  recovery of a known integer translation
# ---------------------------------------------------------------------------
def test_p8_known_translation():
    pair = synth.make_pair("blobs32")
    moving = pair.moving.astype(np.float64)
    fixed = np.roll(moving, -1, axis=2)  # fixed(x) = moving(x + e_x): true u = (1, 0, 0)
    res = O.register(fixed, moving, 0.01, 0.01, 2, 10, 100)
    assert abs(res.disp[0].mean() - 1.0) < 0.05
    gmag = np.sqrt(np.sum(O.gradient(moving) ** 2, axis=0))
    mask = gmag > 0.02
    err = np.sqrt((res.disp[0] - 1.0) ** 2 + res.disp[1] ** 2 + res.disp[2] ** 2)
    assert err[mask].mean() < 0.05


# ---------------------------------------------------------------------------
# P9  adjoints and the sign/scale of the central difference
# ---------------------------------------------------------------------------
def test_p9_gradient_matches_dense_stencil_and_adjoint():
    d = (5, 4, 3)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((3, 4, 5))
    g = O.gradient(f)
    for ax in range(3):
        assert np.allclose(flat(g[ax]), dense_central_diff(d, ax) @ flat(f), atol=1e-14)
    gv = rng.standard_normal((3, 3, 4, 5))
    div = sum(dense_central_diff(d, ax) @ flat(gv[ax]) for ax in range(3))
    assert np.sum(g * gv) == pytest.approx(-np.dot(flat(f), div), rel=1e-12)


def test_p9_gradient_of_plane_wave():
    n = 16
    zz, yy, xx = np.meshgrid(np.arange(8), np.arange(12), np.arange(n), indexing="ij")
    f = np.sin(2 * np.pi * xx / n)
    g = O.gradient(f)
    assert np.allclose(g[0], np.sin(2 * np.pi / n) * np.cos(2 * np.pi * xx / n), atol=1e-14)
    assert np.abs(g[1]).max() == 0 and np.abs(g[2]).max() == 0


def test_p9_rfft_roundtrip_identity():
    rng = np.random.default_rng(2)
    s = rng.standard_normal((3, 6, 4, 8))
    ones = np.ones((6, 4, 5))
    assert np.allclose(O.fourier_solve(s, ones), s, atol=1e-14)


# ---------------------------------------------------------------------------
# P10 Jacobian determinant closed forms
# ---------------------------------------------------------------------------
def test_p10_jacobian_closed_form():
    nx, ny, nz = 16, 8, 6
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    A = 0.8
    u = np.zeros((3, nz, ny, nx))
    u[0] = A * np.sin(2 * np.pi * xx / nx)
    det = O.jacobian_det(u)
    assert np.allclose(det, 1 + A * np.sin(2 * np.pi / nx) * np.cos(2 * np.pi * xx / nx), atol=1e-14)
    u[:] = np.array([0.3, -1.7, 2.2])[:, None, None, None]
    assert np.allclose(O.jacobian_det(u), 1.0, atol=0)
    # a linear map x -> M x (periodic-compatible only through the stencil on
    # interior voxels): det(I + D u) = det(M) away from the wrap-around
    rng = np.random.default_rng(10)
    Mx = rng.uniform(-0.2, 0.2, size=(3, 3))
    coords = np.stack([xx, yy, zz]).astype(np.float64)
    u = np.einsum("cd,d...->c...", Mx, coords)
    det = O.jacobian_det(u)
    assert det[2, 3, 5] == pytest.approx(np.linalg.det(np.eye(3) + Mx), rel=1e-12)
    mn, mx, mean, nneg = O.jacobian_stats(np.zeros((3, 4, 4, 4)))
    assert (mn, mx, mean, nneg) == (1.0, 1.0, 1.0, 0)


# ---------------------------------------------------------------------------
# P11 compose and scaling-and-squaring
# ---------------------------------------------------------------------------
def test_p11_compose_identities():
    d = (10, 8, 6)
    u = synth.random_vector_field(d, seed=4, amp=2.0, smooth_kmax=2).astype(np.float64)
    z = np.zeros_like(u)
    assert np.allclose(O.compose(u, z), u, atol=0)
    assert np.allclose(O.compose(z, u), u, atol=0)
    # integer translations add exactly
    t1 = np.broadcast_to(np.array([2.0, -3.0, 1.0])[:, None, None, None], u.shape).copy()
    t2 = np.broadcast_to(np.array([-5.0, 1.0, 4.0])[:, None, None, None], u.shape).copy()
    assert np.array_equal(O.compose(t1, t2), t1 + t2)
    # composing with an integer shift samples u at the shifted voxel
    c = O.compose(u, t1)
    assert np.allclose(c, t1 + np.roll(u, shift=(-1, 3, -2), axis=(1, 2, 3)), atol=1e-14)
    assert np.allclose(O.expmap(t1 * 0.37, 6), t1 * 0.37, atol=1e-14)


def test_p11_expmap_converges_to_flow():
    """Scaling and squaring approaches the time-1 flow of the stationary field
    (computed independently by RK4 on a cubic-spline field) as K grows."""
    d = (32, 32, 32)
    rng = np.random.default_rng(12)
    vel = 1.5 * synth.band_limited_field(d, rng, kmax=1)
    coeffs = synth.generators._spline_coeffs(vel)
    xx, yy, zz = synth.grid(d)
    ref = synth.flow(coeffs, 1.0, xx, yy, zz, steps=16)
    errs = [np.abs(O.expmap(vel, K) - ref).max() for K in (0, 2, 4, 6)]
    # the error falls with K down to the trilinear interpolation floor
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 0.15 * errs[0] and errs[3] < 0.015 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# P12 trilinear resampling equals SciPy's periodic linear interpolation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("amp", [0.7, 9.3])
def test_p12_trilinear_matches_scipy(amp):
    d = (9, 7, 5)
    rng = np.random.default_rng(13)
    f = rng.standard_normal((5, 7, 9))
    u = amp * rng.standard_normal((3, 5, 7, 9))
    xx, yy, zz = synth.grid(d)
    ref = ndimage.map_coordinates(f, np.stack([(zz + u[2]).ravel(), (yy + u[1]).ravel(), (xx + u[0]).ravel()]),
                                  order=1, mode="grid-wrap").reshape(f.shape)
    assert np.allclose(O.trilinear_periodic(f, u), ref, atol=1e-12)


# ---------------------------------------------------------------------------
# P13 invariants of the iteration and of the whole registration
# ---------------------------------------------------------------------------
def test_p13_iteration_invariants():
    rng = np.random.default_rng(14)
    J = 0.3 * rng.standard_normal((3, 6, 8, 10))
    r = 0.3 * rng.standard_normal((6, 8, 10))
    res = O.admm(J, r, 0.05, 0.1, 2, 12, history=True)
    m = O.w_step_multiplier((10, 8, 6), 0.05, 0.1, 2)
    for h in res.history:
        assert np.abs(h["b"].mean(axis=(1, 2, 3))).max() < 1e-14
    # the w-step never increases the l2 norm (0 < multiplier <= 1)
    s = rng.standard_normal((3, 6, 8, 10))
    assert np.linalg.norm(O.fourier_solve(s, m)) <= np.linalg.norm(s)


def test_p13_registration_equivariance():
    pair = synth.make_pair("blobs32")
    f, mv = pair.fixed.astype(np.float64), pair.moving.astype(np.float64)
    base = O.register(f, mv, 0.01, 0.1, 2, 2, 4)
    # integer periodic roll
    sh = (3, -5, 7)
    rolled = O.register(np.roll(f, sh, axis=(0, 1, 2)), np.roll(mv, sh, axis=(0, 1, 2)), 0.01, 0.1, 2, 2, 4)
    assert np.allclose(rolled.disp, np.roll(base.disp, sh, axis=(1, 2, 3)), atol=1e-12)
    # swapping the x and y axes swaps the x and y displacement components
    ft, mt = np.swapaxes(f, 1, 2), np.swapaxes(mv, 1, 2)
    sw = O.register(ft, mt, 0.01, 0.1, 2, 2, 4)
    expect = np.stack([np.swapaxes(base.disp[1], 1, 2), np.swapaxes(base.disp[0], 1, 2),
                       np.swapaxes(base.disp[2], 1, 2)])
    assert np.allclose(sw.disp, expect, atol=1e-12)


# ---------------------------------------------------------------------------
# P14 positivity of the Jacobian on the 32^3 blob workload
# ---------------------------------------------------------------------------
def test_p14_blob_workload_is_diffeomorphic_and_improves():
    pair = synth.make_pair("blobs32")
    w = synth.WORKLOADS["blobs32"]
    res = O.register(pair.fixed, pair.moving, w["lam"], w["theta"], w["order"], w["outer"], w["iters"])
    mn, mx, mean, nneg = O.jacobian_stats(res.disp)
    assert nneg == 0 and mn > 0
    assert O.ssd(pair.fixed, res.warped) < 0.1 * O.ssd(pair.fixed, pair.moving)


# ---------------------------------------------------------------------------
# P15 the un-restarted accelerated iteration can diverge (documented)
# ---------------------------------------------------------------------------
def test_p15_divergence_is_visible_in_residuals():
    rng = np.random.default_rng(15)
    J = rng.choice([-1.0, 1.0], size=(3, 4, 4, 4)) / math.sqrt(3)  # |J| = 1
    r = rng.uniform(-0.5, 0.5, size=(4, 4, 4))
    with np.errstate(all="ignore"):
        res = O.admm(J, r, 10.0, 0.1, 1, 200, history=True)
    p = np.array([h["primal"] for h in res.history])
    assert not np.isfinite(p[-1]) or p[-1] > 10 * p[:50].min()
    # the safe regime (small |J| and lambda) converges
    res2 = O.admm(0.3 * J, r, 0.5, 0.1, 1, 200, history=True)
    p2 = np.array([h["primal"] for h in res2.history])
    assert p2[-1] < 1e-8 * p2[0]


def test_p15b_divergence_guard():
    """The guard (no rule in the paper; the reading: after K >= 3 iterations
    the last fixed-point residual |s^{K-1} - s^{K-2}| exceeds the first
    |s^1 - s^0|) recomputed from the recorded iterates, s^k = w^k + b^k: set
    in the divergent regime of P15, clear in its safe regime and for K < 3."""
    rng = np.random.default_rng(15)
    J = rng.choice([-1.0, 1.0], size=(3, 4, 4, 4)) / math.sqrt(3)
    r = rng.uniform(-0.5, 0.5, size=(4, 4, 4))

    def from_history(res):
        s = [h["w"] + h["b"] for h in res.history]
        first = np.sum((s[1] - s[0]) ** 2)
        last = np.sum((s[-1] - s[-2]) ** 2)
        return bool(not np.isfinite(last) or last > first)

    with np.errstate(all="ignore"):
        bad = O.admm(J, r, 10.0, 0.1, 1, 60, history=True)
    assert bad.diverged and from_history(bad)
    good = O.admm(0.3 * J, r, 0.5, 0.1, 1, 60, history=True)
    assert not good.diverged and not from_history(good)
    for k in (1, 2):
        with np.errstate(all="ignore"):
            assert not O.admm(J, r, 10.0, 0.1, 1, k).diverged
    # registration: one flag per warping
    d = (8, 6, 4)
    f = synth.random_volume(d, seed=150).astype(np.float64)
    m = synth.random_volume(d, seed=151).astype(np.float64)
    reg = O.register(f, m, 0.01, 0.1, 2, 2, 6)
    assert reg.diverged == [False, False]


# ---------------------------------------------------------------------------
# P16-P19: the adjoint of one warping (reverse mode through Eq. (5), (6))
# ---------------------------------------------------------------------------
def _smooth(d, seed):
    return synth.random_volume(d, seed=seed, smooth_kmax=2).astype(np.float64)


def test_p16_warp_transpose_is_adjoint():
    d = (7, 6, 5)
    rng = np.random.default_rng(160)
    f = rng.standard_normal(d[::-1])
    g = rng.standard_normal(d[::-1])
    u = 2.5 * rng.standard_normal((3,) + d[::-1])
    lhs = np.sum(O.trilinear_periodic(f, u) * g)
    rhs = np.sum(f * O.trilinear_transpose(g, u))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_p17_position_gradient_matches_differences():
    d = (8, 7, 6)
    rng = np.random.default_rng(170)
    f = rng.standard_normal(d[::-1])
    u = 1.7 * rng.standard_normal((3,) + d[::-1])
    # stay away from cell faces, where the one-sided derivative jumps
    frac = u - np.floor(u)
    u = np.floor(u) + np.clip(frac, 0.05, 0.95)
    grad = O.trilinear_position_gradient(f, u)
    h = 1e-6
    for c in range(3):
        e = np.zeros_like(u)
        e[c] = h
        fd = (O.trilinear_periodic(f, u + e) - O.trilinear_periodic(f, u - e)) / (2 * h)
        assert np.abs(fd - grad[c]).max() < 1e-7


def test_p18_data_step_adjoint_matches_differences():
    rng = np.random.default_rng(180)
    shp = (3, 4, 3, 5)
    a, J, gv = (rng.standard_normal(shp) for _ in range(3))
    r = rng.standard_normal(shp[1:])
    theta = 0.3
    ga, gJ, gr = O.v_step_l2_adjoint(gv, a, J, r, theta)
    h = 1e-6
    for x, gx in ((a, ga), (J, gJ)):
        dx = rng.standard_normal(shp)
        pa = O.v_step_l2(a + h * dx if x is a else a, J + h * dx if x is J else J, r, theta)
        ma = O.v_step_l2(a - h * dx if x is a else a, J - h * dx if x is J else J, r, theta)
        fd = np.sum(gv * (pa - ma)) / (2 * h)
        assert abs(fd - np.sum(gx * dx)) < 1e-7 * max(1.0, abs(fd))
    dr = rng.standard_normal(shp[1:])
    fd = np.sum(gv * (O.v_step_l2(a, J, r + h * dr, theta) - O.v_step_l2(a, J, r - h * dr, theta))) / (2 * h)
    assert abs(fd - np.sum(gr * dr)) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("order,iters", [(1, 3), (2, 6)])
def test_p19_one_warping_gradient_matches_differences(order, iters):
    d = (10, 8, 6)
    f = _smooth(d, 190)
    m = _smooth(d, 191)
    lam, theta = 0.05, 0.1
    loss, gm, gl = O.ssd_one_warping_grad(f, m, lam, theta, order, iters)
    assert abs(loss - O.ssd_one_warping(f, m, lam, theta, order, iters)) < 1e-12 * loss
    rng = np.random.default_rng(192)
    h = 1e-6
    for _ in range(6):
        i = tuple(int(rng.integers(0, n)) for n in m.shape)
        mp, mm = m.copy(), m.copy()
        mp[i] += h
        mm[i] -= h
        fd = (O.ssd_one_warping(f, mp, lam, theta, order, iters)
              - O.ssd_one_warping(f, mm, lam, theta, order, iters)) / (2 * h)
        assert abs(fd - gm[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, gm[i])
    fd = (O.ssd_one_warping(f, m, lam + h, theta, order, iters)
          - O.ssd_one_warping(f, m, lam - h, theta, order, iters)) / (2 * h)
    assert abs(fd - gl) < 1e-6 * max(1.0, abs(fd)), (fd, gl)


# ---------------------------------------------------------------------------
# P20: the pyramid's resampling
# ---------------------------------------------------------------------------
def test_p20_pyramid_resampling():
    rng = np.random.default_rng(200)
    # averaging: block-constant volumes come back exactly, means are kept
    blocks = rng.standard_normal((3, 4, 5))
    f = np.repeat(np.repeat(np.repeat(blocks, 2, 0), 2, 1), 2, 2)
    assert np.array_equal(O.downsample2(f), blocks)
    g = rng.standard_normal((6, 8, 10))
    assert abs(O.downsample2(g).mean() - g.mean()) < 1e-14
    # the general sampler equals the library's periodic linear interpolation
    c = rng.standard_normal((5, 6, 7))
    pts = [rng.uniform(-8, 16, 50) for _ in range(3)]
    ref = ndimage.map_coordinates(c, np.stack([pts[2], pts[1], pts[0]]), order=1, mode="grid-wrap")
    assert np.abs(O.sample_periodic(c, *pts) - ref).max() < 1e-12
    # carrying a displacement: constants double
    const = np.stack([np.full((4, 5, 6), v) for v in (0.5, -1.25, 2.0)])
    up = O.upsample2_disp(const)
    assert up.shape == (3, 8, 10, 12)
    assert np.allclose(up[0], 1.0) and np.allclose(up[1], -2.5) and np.allclose(up[2], 4.0)
    # a profile along x only: fine voxel 2i samples coarse position i - 1/4 and
    # 2i + 1 samples i + 1/4, so u_f(2i) = 2 (u(i-1)/4 + 3 u(i)/4) and
    # u_f(2i+1) = 2 (3 u(i)/4 + u(i+1)/4), indices periodic
    prof = rng.standard_normal(6)
    u = np.zeros((3, 4, 5, 6))
    u[1] = prof[None, None, :]
    upu = O.upsample2_disp(u)[1, 0, 0]
    prev, nxt = np.roll(prof, 1), np.roll(prof, -1)
    assert np.abs(upu[0::2] - 2.0 * (0.25 * prev + 0.75 * prof)).max() < 1e-12
    assert np.abs(upu[1::2] - 2.0 * (0.75 * prof + 0.25 * nxt)).max() < 1e-12


def test_p20_pyramid_identity_and_levels():
    d = (32, 24, 16)
    img = synth.random_volume(d, seed=201, smooth_kmax=2).astype(np.float64)
    res = O.pyramid_register(img, img, 0.01, 0.1, 2, outer=(2, 2, 1), iters=(3, 2, 2))
    assert np.array_equal(res.disp, np.zeros_like(res.disp))
    # one level is a plain registration
    f = synth.random_volume(d, seed=202, smooth_kmax=2).astype(np.float64)
    one = O.pyramid_register(f, img, 0.01, 0.1, 2, outer=(2,), iters=(3,))
    ref = O.register(f, img, 0.01, 0.1, 2, 2, 3)
    assert np.array_equal(one.disp, ref.disp)


# ---------------------------------------------------------------------------
# P21: threshold stopping (Sec. 4, second hyperparameter version)
# ---------------------------------------------------------------------------
def test_p21_admm_threshold_stops_at_first_crossing():
    rng = np.random.default_rng(210)
    J = 0.3 * rng.standard_normal((3, 6, 8, 10))
    r = 0.3 * rng.standard_normal((6, 8, 10))
    lam, theta, order, cap = 0.05, 0.1, 2, 14
    full = O.admm(J, r, lam, theta, order, cap, history=True)
    # the w-step input s^k = v^k + b_hat^k equals w^k + b^k (b^k = b_hat^k + v^k - w^k):
    # its relative change, from the recorded w and b
    s = [h["w"] + h["b"] for h in full.history]
    rho = [np.linalg.norm(s[k] - s[k - 1]) / np.linalg.norm(s[k]) for k in range(1, cap)]
    traced = O.admm(J, r, lam, theta, order, cap, tol=0.0)
    assert traced.iters_run == cap
    assert np.allclose(traced.rel_change, rho, rtol=1e-12, atol=0)
    for pick in (2, 6, 9):
        tol = 1.001 * rho[pick]
        k_stop = next(k for k in range(1, cap) if rho[k - 1] <= tol)
        res = O.admm(J, r, lam, theta, order, cap, tol=tol)
        assert res.iters_run == k_stop + 1
        assert np.array_equal(res.w, O.admm(J, r, lam, theta, order, k_stop + 1).w)
    # a threshold above every change stops after the first check (k = 1)
    assert O.admm(J, r, lam, theta, order, cap, tol=1e30).iters_run == 2
    # zero data term: s stays exactly zero, which meets any threshold
    z = O.admm(J, np.zeros_like(r), lam, theta, order, cap, tol=0.0)
    assert z.iters_run == 2 and not z.w.any()


def test_p21_warping_threshold_stops_at_first_crossing():
    pair = synth.make_pair("blobs32")
    f, mv = pair.fixed.astype(np.float64), pair.moving.astype(np.float64)
    lam, theta, order, outer, iters = 0.01, 0.1, 2, 5, 4
    # u_c for c = 0 .. outer-1 by plain registrations of c + 1 warpings
    us = [O.register(f, mv, lam, theta, order, c + 1, iters).disp for c in range(outer)]
    delta = [np.linalg.norm(us[c] - us[c - 1]) / np.linalg.norm(us[c]) for c in range(1, outer)]
    traced = O.register(f, mv, lam, theta, order, outer, iters, tol_warp=0.0)
    assert np.allclose(traced.warp_change, delta, rtol=1e-12, atol=0)
    assert np.array_equal(traced.disp, us[-1])
    for pick in (0, 2):
        tol = 1.001 * delta[pick]
        c_stop = next(c for c in range(1, outer) if delta[c - 1] <= tol)
        res = O.register(f, mv, lam, theta, order, outer, iters, tol_warp=tol)
        assert len(res.iters_run) == c_stop + 1
        assert np.array_equal(res.disp, us[c_stop])
        assert np.array_equal(res.warped, O.trilinear_periodic(mv, us[c_stop]))
    # identical images: every field is exactly zero, both loops stop at their first check
    same = O.register(mv, mv, lam, theta, order, outer, iters, tol_admm=0.0, tol_warp=0.0)
    assert same.iters_run == [2, 2] and not same.disp.any()


def test_p21_pyramid_with_thresholds():
    d = (32, 24, 16)
    f = synth.random_volume(d, seed=211, smooth_kmax=2).astype(np.float64)
    m = synth.random_volume(d, seed=212, smooth_kmax=2).astype(np.float64)
    outer, iters = (3, 3, 2), (4, 3, 3)
    plain = O.pyramid_register(f, m, 0.01, 0.1, 2, outer, iters)
    # thresholds no change reaches: the capped schedule, bit for bit
    never = O.pyramid_register(f, m, 0.01, 0.1, 2, outer, iters, tol_admm=0.0, tol_warp=0.0)
    assert np.array_equal(never.disp, plain.disp)
    assert never.level_iters == [[4, 4, 4], [3, 3, 3], [3, 3]]
    # thresholds every change meets: two warpings of two iterations per level
    first = O.pyramid_register(f, m, 0.01, 0.1, 2, outer, iters, tol_admm=1e30, tol_warp=1e30)
    assert first.level_iters == [[2, 2], [2, 2], [2, 2]]
    ref = O.pyramid_register(f, m, 0.01, 0.1, 2, (2, 2, 2), (2, 2, 2))
    assert np.array_equal(first.disp, ref.disp)
