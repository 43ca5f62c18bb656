"""Plain FP64 CPU oracle for Nesterov-accelerated ADMM diffeomorphic registration.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and it
shares no code, tables or constants with that path.

Everything here follows the paper (Thorley et al., "Nesterov Accelerated ADMM
for Fast Diffeomorphic Image Registration") step by step, in NumPy float64,
with no blocking, fusion or reordering beyond what the paper states:

* Sec. 2, Eq. (1) with N = 1: the deformation is the composition of the
  per-warping velocity fields, and the *original* source image is warped by
  the whole composition each time (Sec. 2, the iterative scheme).
* Sec. 2, Eq. (2) with s = 2: the linearised data term
  rho(v) = <grad I1, v> + I1 - I0 and the order-n regulariser.
* Sec. 3, Eq. (3)-(5): variable splitting w = v, scaled augmented Lagrangian
  and the Nesterov-accelerated ADMM recurrence, including the alpha/gamma
  momentum scalars and the zero initialisation.
* Sec. 3, Eq. (6): the closed-form v-step (Sherman-Morrison, s = 2) and the
  Fourier-diagonalised w-step with the finite-difference symbol of the
  Laplacian.

Readings of points the paper leaves open (each is listed in the design notes):

* The w-step is read with theta in the numerator,
  w = F^-1( theta F(v + b_hat) / (theta + lambda F(Delta^n)) ): that is the
  optimality condition of the w-subproblem of Eq. (5); the printed Eq. (6)
  omits the factor.
* F(Delta^n) is the (non-negative) symbol of (-Delta_h)^n for the 7-point
  periodic Laplacian with unit spacing, as printed in Sec. 3.
* grad I1 is the periodic central difference (unit spacing) of the warped
  source image passed to the model (Sec. 2).
* Warps and compositions use periodic trilinear interpolation (floor of the
  sample position, indices taken modulo the size).
* Each warping starts the ADMM loop from zero with alpha^0 = 1 (Sec. 3, text
  after Eq. (5)); the warping's velocity is the final w iterate.
* Loop counts are fixed (Sec. 4, first hyperparameter version caps them).
  Optionally (Sec. 4, second hyperparameter version) the loops stop at
  thresholds whose measures the paper does not define.  Readings: the ADMM
  loop stops after iteration k >= 1 once |s^k - s^{k-1}| <= tol |s^k|, with
  s^k = v^k + b_hat^k the input of the w-step and |.| the L2 norm over the
  whole vector field; the warping loop stops after warping c >= 1 (0-based:
  from the second warping on) once |u_c - u_{c-1}| <= tol |u_c|.  Both
  loops keep their caps.  A stopped ADMM loop returns the w^k of the
  iteration that met the threshold.

Array conventions: scalar volumes have shape (nz, ny, nx) with x fastest;
vector fields have shape (3, nz, ny, nx) with component 0 the x displacement,
1 the y and 2 the z displacement, in voxel units.  Displacements are
backward (pull): the warped image is I(x + u(x)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

AXIS_OF_COMPONENT = (2, 1, 0)  # numpy axis that carries x, y, z


# ---------------------------------------------------------------------------
# Nesterov scalars -- Sec. 3, Eq. (5)
# ---------------------------------------------------------------------------
def nesterov_alphas(iters: int) -> np.ndarray:
    """alpha^0 .. alpha^iters of Eq. (5): alpha^0 = 1 and
    alpha^{k+1} = (1 + sqrt(1 + 4 (alpha^k)^2)) / 2."""
    a = np.empty(iters + 1, dtype=np.float64)
    a[0] = 1.0
    for k in range(iters):
        a[k + 1] = (1.0 + math.sqrt(1.0 + 4.0 * a[k] * a[k])) / 2.0
    return a


def nesterov_gammas(iters: int) -> np.ndarray:
    """gamma_k = (alpha^k - 1) / alpha^{k+1}, the extrapolation weight that
    builds w_hat^{k+1}, b_hat^{k+1} from iterates k and k-1 (Eq. (5))."""
    a = nesterov_alphas(iters)
    return (a[:-1] - 1.0) / a[1:]


# ---------------------------------------------------------------------------
# Finite differences and the Laplacian symbol -- Sec. 3, text after Eq. (6)
# ---------------------------------------------------------------------------
def central_diff(f: np.ndarray, axis: int) -> np.ndarray:
    """Periodic central difference with unit spacing along a numpy axis."""
    return (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)) / 2.0


def gradient(f: np.ndarray) -> np.ndarray:
    """(d/dx, d/dy, d/dz) of a scalar volume, periodic central differences."""
    return np.stack([central_diff(f, ax) for ax in AXIS_OF_COMPONENT])


def laplacian_symbol(dims_xyz, half: bool = True) -> np.ndarray:
    """2 (3 - cos(2 pi p/M) - cos(2 pi q/N) - cos(2 pi r/H)) on the DFT grid,
    i.e. the eigenvalues of the periodic 7-point -Delta_h (Sec. 3).

    Returned with shape (nz, ny, nx//2+1) when ``half`` (the real-FFT half
    grid of numpy.fft.rfftn over axes (0, 1, 2)), else (nz, ny, nx)."""
    nx, ny, nz = dims_xyz
    px = np.arange(nx // 2 + 1 if half else nx)
    q = np.arange(ny)
    r = np.arange(nz)
    cx = np.cos(2.0 * np.pi * px / nx)[None, None, :]
    cy = np.cos(2.0 * np.pi * q / ny)[None, :, None]
    cz = np.cos(2.0 * np.pi * r / nz)[:, None, None]
    return 2.0 * (3.0 - cx - cy - cz)


def w_step_multiplier(dims_xyz, lam: float, theta: float, order: int,
                      half: bool = True) -> np.ndarray:
    """theta / (theta + lambda * F(Delta^n)) with F(Delta^n) = symbol**n."""
    k = laplacian_symbol(dims_xyz, half=half) ** order
    return theta / (theta + lam * k)


def fourier_solve(s: np.ndarray, mult: np.ndarray) -> np.ndarray:
    """w = F^-1( mult * F(s) ) per component (w-step of Eq. (6)).

    F is the unnormalised forward DFT, F^-1 its inverse (numpy convention)."""
    shape = s.shape[-3:]
    out = np.empty_like(s)
    for c in range(s.shape[0]):
        out[c] = np.fft.irfftn(mult * np.fft.rfftn(s[c], axes=(0, 1, 2)), s=shape, axes=(0, 1, 2))
    return out


# ---------------------------------------------------------------------------
# Periodic trilinear resampling -- Sec. 2 (warping I1 by Id + v)
# ---------------------------------------------------------------------------
def trilinear_periodic(f: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """Sample f at x + disp(x) for every voxel x, trilinear, periodic.

    f: (nz, ny, nx) scalar, or (C, nz, ny, nx) stacked scalars sampled at the
    same points.  disp: (3, nz, ny, nx) in voxels (component 0 = x)."""
    nz, ny, nx = disp.shape[1:]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    px = xx + disp[0]
    py = yy + disp[1]
    pz = zz + disp[2]
    fx = np.floor(px)
    fy = np.floor(py)
    fz = np.floor(pz)
    tx = px - fx
    ty = py - fy
    tz = pz - fz
    ix0 = np.mod(fx.astype(np.int64), nx)
    iy0 = np.mod(fy.astype(np.int64), ny)
    iz0 = np.mod(fz.astype(np.int64), nz)
    ix1 = np.mod(ix0 + 1, nx)
    iy1 = np.mod(iy0 + 1, ny)
    iz1 = np.mod(iz0 + 1, nz)

    def one(g):
        return ((1 - tz) * ((1 - ty) * ((1 - tx) * g[iz0, iy0, ix0] + tx * g[iz0, iy0, ix1])
                            + ty * ((1 - tx) * g[iz0, iy1, ix0] + tx * g[iz0, iy1, ix1]))
                + tz * ((1 - ty) * ((1 - tx) * g[iz1, iy0, ix0] + tx * g[iz1, iy0, ix1])
                        + ty * ((1 - tx) * g[iz1, iy1, ix0] + tx * g[iz1, iy1, ix1])))

    if f.ndim == 3:
        return one(f)
    return np.stack([one(f[c]) for c in range(f.shape[0])])


def compose(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Displacement of (Id + u) o (Id + v):  v(x) + u(x + v(x))  (Eq. (1))."""
    return v + trilinear_periodic(u, v)


def expmap(vel: np.ndarray, steps: int) -> np.ndarray:
    """Scaling and squaring of a stationary velocity field: u = vel / 2^K,
    then K self-compositions u <- u + u(x + u(x))."""
    u = vel / float(2 ** steps)
    for _ in range(steps):
        u = compose(u, u)
    return u


# ---------------------------------------------------------------------------
# Data term and the closed-form v-step -- Sec. 2 Eq. (2), Sec. 3 Eq. (6)
# ---------------------------------------------------------------------------
def warp_grad_residual(moving: np.ndarray, fixed: np.ndarray, disp: np.ndarray):
    """I1^w = I1 o (Id + disp);  J = grad I1^w;  r = I1^w - I0.

    The linearised residual of Eq. (2) is then rho(v) = <J, v> + r."""
    warped = trilinear_periodic(moving, disp)
    return warped, gradient(warped), warped - fixed


def v_step_l2(a: np.ndarray, J: np.ndarray, r: np.ndarray, theta: float) -> np.ndarray:
    """Solve (J J^T + theta I) v = theta a - J r per voxel (Eq. (6), s = 2),
    with a = w_hat - b_hat.  By Sherman-Morrison for the rank-one J J^T:
    v = a - J (J.a + r) / (theta + |J|^2)."""
    ja = np.sum(J * a, axis=0)
    jj = np.sum(J * J, axis=0)
    return a - J * ((ja + r) / (theta + jj))[None]


def v_step_l1(a: np.ndarray, J: np.ndarray, r: np.ndarray, theta: float,
              eps: float = 1e-8) -> np.ndarray:
    """Eq. (6), s = 1: v = a - z_hat / max(|z_hat|, 1) * J / theta with
    z_hat = theta rho(a) / (|J|^2 + eps)."""
    rho = np.sum(J * a, axis=0) + r
    z = theta * rho / (np.sum(J * J, axis=0) + eps)
    return a - (z / np.maximum(np.abs(z), 1.0))[None] * J / theta


# ---------------------------------------------------------------------------
# Nesterov-accelerated ADMM -- Sec. 3, Eq. (5) and (6)
# ---------------------------------------------------------------------------
@dataclass
class AdmmResult:
    w: np.ndarray
    b: np.ndarray
    v: np.ndarray
    gammas: np.ndarray
    history: list = field(default_factory=list)
    iters_run: int = 0
    rel_change: list = field(default_factory=list)  # |s^k - s^{k-1}| / |s^k|, k >= 1
    # divergence guard: |s^{K-1} - s^{K-2}| > |s^1 - s^0| after K >= 3 iterations
    diverged: bool = False


def rel_change(new: np.ndarray, old: np.ndarray) -> float:
    """|new - old| / |new| in the L2 norm over the whole field (0 when both
    are zero, inf when only new is)."""
    d, n = float(np.sum((new - old) ** 2)), float(np.sum(new ** 2))
    if n > 0:
        return math.sqrt(d / n)
    return 0.0 if d == 0 else math.inf


def below_threshold(new: np.ndarray, old: np.ndarray, tol: float) -> bool:
    """|new - old| <= tol |new| (squared on both sides; true when both are 0)."""
    return float(np.sum((new - old) ** 2)) <= tol * tol * float(np.sum(new ** 2))


def admm(J: np.ndarray, r: np.ndarray, lam: float, theta: float, order: int,
         iters: int, data_term: int = 2, eps: float = 1e-8,
         history: bool = False, mult: np.ndarray | None = None,
         tol: float | None = None) -> AdmmResult:
    """Run ``iters`` iterations (k = 0 .. iters-1) of Eq. (5) from the
    initialisation w_hat^0 = b_hat^0 = 0, alpha^0 = 1.

    Per iteration, in the paper's order:
      v^k = argmin of the data subproblem          (Eq. (6), top/middle)
      w^k = F^-1( theta F(v^k + b_hat^k) / (theta + lambda F(Delta^n)) )
      b^k = b_hat^k + v^k - w^k
      alpha^{k+1} = (1 + sqrt(1 + 4 (alpha^k)^2)) / 2
      w_hat^{k+1} = w^k + (alpha^k - 1)/alpha^{k+1} (w^k - w^{k-1})
      b_hat^{k+1} = b^k + (alpha^k - 1)/alpha^{k+1} (b^k - b^{k-1})
    ``mult`` overrides the w-step multiplier (used only by tests that plant a
    mistake to show the pins catch it).  With ``tol`` the loop also stops
    after the first iteration k >= 1 whose w-step input s^k = v^k + b_hat^k
    satisfies |s^k - s^{k-1}| <= tol |s^k| (threshold stopping, Sec. 4).

    ``diverged`` (the paper gives no restart or divergence rule; this is the
    guard's reading): after K >= 3 iterations, the fixed-point residual of
    the last iteration exceeds that of the first, |s^{K-1} - s^{K-2}| >
    |s^1 - s^0| in the L2 norm over the whole field (or is not finite)."""
    dims_xyz = (J.shape[3], J.shape[2], J.shape[1])
    if mult is None:
        mult = w_step_multiplier(dims_xyz, lam, theta, order)
    zeros = np.zeros_like(J)
    w_hat, b_hat = zeros.copy(), zeros.copy()
    w_prev, b_prev = zeros.copy(), zeros.copy()  # w^{-1}, b^{-1}
    alpha = 1.0
    gam = []
    hist = []
    w = b = v = zeros
    s_prev = None
    changes = []
    stop = False
    k_run = 0
    first_res = 0.0
    diverged = False
    for k in range(iters):
        a = w_hat - b_hat
        if data_term == 2:
            v = v_step_l2(a, J, r, theta)
        else:
            v = v_step_l1(a, J, r, theta, eps)
        s = v + b_hat
        w = fourier_solve(s, mult)
        b = b_hat + v - w
        k_run = k + 1
        if tol is not None and s_prev is not None:
            changes.append(rel_change(s, s_prev))
            stop = below_threshold(s, s_prev, tol)
        if k == 1:
            first_res = float(np.sum((s - s_prev) ** 2))
        if k == iters - 1 and k >= 2:
            last_res = float(np.sum((s - s_prev) ** 2))
            diverged = not math.isfinite(last_res) or last_res > first_res
        s_prev = s
        alpha_next = (1.0 + math.sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0
        g = (alpha - 1.0) / alpha_next
        gam.append(g)
        if history:
            # primal residual |w^k - v^k| and dual residual theta |w^k - w^{k-1}|
            hist.append({"v": v.copy(), "w": w.copy(), "b": b.copy(),
                         "primal": float(np.sqrt(np.sum((w - v) ** 2))),
                         "dual": float(theta * np.sqrt(np.sum((w - w_prev) ** 2)))})
        if stop:
            break
        w_hat = w + g * (w - w_prev)
        b_hat = b + g * (b - b_prev)
        w_prev, b_prev = w, b
        alpha = alpha_next
    return AdmmResult(w=w, b=b, v=v, gammas=np.array(gam), history=hist, iters_run=k_run,
                      rel_change=changes, diverged=diverged and k_run == iters)


# ---------------------------------------------------------------------------
# Outer composition loop -- Sec. 2, Eq. (1) with N = 1
# ---------------------------------------------------------------------------
@dataclass
class RegisterResult:
    disp: np.ndarray
    warped: np.ndarray
    velocities: list
    iters_run: list = field(default_factory=list)     # ADMM iterations of each warping
    level_iters: list = field(default_factory=list)   # pyramid: iters_run of every level
    admm_change: list = field(default_factory=list)   # per warping: its ADMM rel_change list
    warp_change: list = field(default_factory=list)   # |u_c - u_{c-1}| / |u_c|, c >= 1
    diverged: list = field(default_factory=list)      # the ADMM guard of each warping


def register(fixed: np.ndarray, moving: np.ndarray, lam: float, theta: float,
             order: int, outer: int, iters: int, data_term: int = 2,
             init_disp: np.ndarray | None = None,
             keep_velocities: bool = False,
             tol_admm: float | None = None, tol_warp: float | None = None) -> RegisterResult:
    """The iterative scheme of Sec. 2: solve the model for a velocity with
    the current warped source, compose it onto the deformation, warp the
    original source again, repeat ``outer`` times.

    Composition order (Sec. 2): phi_c = phi_{c-1} o (Id + v_c), so the
    displacement becomes u_c(x) = v_c(x) + u_{c-1}(x + v_c(x)).

    ``tol_admm`` / ``tol_warp`` add the threshold stopping of Sec. 4's second
    hyperparameter version (see ``admm``; the warping loop stops after
    warping c >= 1 once |u_c - u_{c-1}| <= tol_warp |u_c|)."""
    fixed = np.asarray(fixed, dtype=np.float64)
    moving = np.asarray(moving, dtype=np.float64)
    u = np.zeros((3,) + fixed.shape) if init_disp is None else np.asarray(init_disp, np.float64).copy()
    vels, runs, achg, wchg, divs = [], [], [], [], []
    for c in range(outer):
        _, J, r = warp_grad_residual(moving, fixed, u)
        res = admm(J, r, lam, theta, order, iters, data_term=data_term, tol=tol_admm)
        runs.append(res.iters_run)
        achg.append(res.rel_change)
        divs.append(res.diverged)
        vel = res.w
        if keep_velocities:
            vels.append(vel.copy())
        u_prev, u = u, compose(u, vel)
        if tol_warp is not None and c >= 1:
            wchg.append(rel_change(u, u_prev))
            if below_threshold(u, u_prev, tol_warp):
                break
    warped = trilinear_periodic(moving, u)
    return RegisterResult(disp=u, warped=warped, velocities=vels, iters_run=runs, admm_change=achg,
                          warp_change=wchg, diverged=divs)


# ---------------------------------------------------------------------------
# Jacobian-determinant check -- Sec. 4 (percentage of non-positive |J_phi|)
# ---------------------------------------------------------------------------
def jacobian_det(disp: np.ndarray) -> np.ndarray:
    """det(I + D u) per voxel, D by periodic central differences."""
    D = np.empty((3, 3) + disp.shape[1:])
    for c in range(3):
        for d in range(3):
            D[c, d] = central_diff(disp[c], AXIS_OF_COMPONENT[d])
    A = D + np.eye(3)[:, :, None, None, None]
    return (A[0, 0] * (A[1, 1] * A[2, 2] - A[1, 2] * A[2, 1])
            - A[0, 1] * (A[1, 0] * A[2, 2] - A[1, 2] * A[2, 0])
            + A[0, 2] * (A[1, 0] * A[2, 1] - A[1, 1] * A[2, 0]))


def jacobian_stats(disp: np.ndarray):
    """(min det, max det, mean det, number of voxels with det <= 0)."""
    d = jacobian_det(disp)
    return float(d.min()), float(d.max()), float(d.mean()), int(np.count_nonzero(d <= 0))


def ssd(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.sum((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))


# ---------------------------------------------------------------------------
# Differentiation of one warping (reverse mode through Sec. 3, Eq. (5), (6))
# ---------------------------------------------------------------------------
# The loss is the SSD between the fixed image and the moving image warped by
# the velocity of ONE warping from u = 0 (Sec. 2, the first pass of the
# iterative scheme), i.e. L = sum (I1(x + w(x)) - I0(x))^2 with w the final
# ADMM iterate of Eq. (5) for J = grad I1, r = I1 - I0.  The gradients with
# respect to I1 and lambda are taken by reverse-mode differentiation of the
# recurrence exactly as `admm` runs it, each step's adjoint written out:
#   a = w_hat - b_hat;  v = D(a);  s = v + b_hat;  w = S s;  b = s - w;
#   w_hat' = w + gamma (w - w_prev);  b_hat' = b + gamma (b - b_prev).
# S is real-symmetric in the Fourier basis (S^T = S) and
# dS/dlambda = F^-1 [ -theta K^n / (theta + lambda K^n)^2 ] F.

def trilinear_transpose(g: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """W^T g for the warp W f = trilinear_periodic(f, disp): each voxel's
    value g(x) is added to the 8 grid points around x + disp(x) with the
    trilinear weights (so <W f, g> = <f, W^T g>)."""
    nz, ny, nx = disp.shape[1:]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    px, py, pz = xx + disp[0], yy + disp[1], zz + disp[2]
    fx, fy, fz = np.floor(px), np.floor(py), np.floor(pz)
    tx, ty, tz = px - fx, py - fy, pz - fz
    ix0 = np.mod(fx.astype(np.int64), nx)
    iy0 = np.mod(fy.astype(np.int64), ny)
    iz0 = np.mod(fz.astype(np.int64), nz)
    out = np.zeros((nz, ny, nx))
    for dz, wz in ((0, 1 - tz), (1, tz)):
        for dy, wy in ((0, 1 - ty), (1, ty)):
            for dx, wx in ((0, 1 - tx), (1, tx)):
                np.add.at(out, (np.mod(iz0 + dz, nz), np.mod(iy0 + dy, ny), np.mod(ix0 + dx, nx)),
                          wz * wy * wx * g)
    return out


def trilinear_position_gradient(f: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """d/dp of the trilinear interpolant of f at p = x + disp(x), per axis
    (the one-sided derivative at integer positions, where the floor is
    taken): shape (3, nz, ny, nx)."""
    nz, ny, nx = disp.shape[1:]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    px, py, pz = xx + disp[0], yy + disp[1], zz + disp[2]
    fx, fy, fz = np.floor(px), np.floor(py), np.floor(pz)
    tx, ty, tz = px - fx, py - fy, pz - fz
    x0 = np.mod(fx.astype(np.int64), nx)
    y0 = np.mod(fy.astype(np.int64), ny)
    z0 = np.mod(fz.astype(np.int64), nz)
    x1, y1, z1 = np.mod(x0 + 1, nx), np.mod(y0 + 1, ny), np.mod(z0 + 1, nz)
    c = {(i, j, k): f[(z0, z1)[k], (y0, y1)[j], (x0, x1)[i]]
         for i in (0, 1) for j in (0, 1) for k in (0, 1)}
    gx = ((1 - ty) * (1 - tz) * (c[1, 0, 0] - c[0, 0, 0]) + ty * (1 - tz) * (c[1, 1, 0] - c[0, 1, 0])
          + (1 - ty) * tz * (c[1, 0, 1] - c[0, 0, 1]) + ty * tz * (c[1, 1, 1] - c[0, 1, 1]))
    gy = ((1 - tx) * (1 - tz) * (c[0, 1, 0] - c[0, 0, 0]) + tx * (1 - tz) * (c[1, 1, 0] - c[1, 0, 0])
          + (1 - tx) * tz * (c[0, 1, 1] - c[0, 0, 1]) + tx * tz * (c[1, 1, 1] - c[1, 0, 1]))
    gz = ((1 - tx) * (1 - ty) * (c[0, 0, 1] - c[0, 0, 0]) + tx * (1 - ty) * (c[1, 0, 1] - c[1, 0, 0])
          + (1 - tx) * ty * (c[0, 1, 1] - c[0, 1, 0]) + tx * ty * (c[1, 1, 1] - c[1, 1, 0]))
    return np.stack([gx, gy, gz])


def v_step_l2_adjoint(gv: np.ndarray, a: np.ndarray, J: np.ndarray, r: np.ndarray,
                      theta: float):
    """Transpose of the Jacobian of v = a - J (J.a + r) / (theta + |J|^2)
    applied to gv: returns (ga, gJ, gr).  With q = theta + |J|^2 and
    f = (J.a + r) / q:  dv/da = I - J J^T / q (symmetric),  dv/dr = -J / q,
    dv_i/dJ_j = -delta_ij f - J_i (a_j - 2 f J_j) / q."""
    q = theta + np.sum(J * J, axis=0)
    f = (np.sum(J * a, axis=0) + r) / q
    jg = np.sum(J * gv, axis=0)
    ga = gv - J * (jg / q)[None]
    gr = -jg / q
    gJ = -f[None] * gv - (jg / q)[None] * (a - 2.0 * f[None] * J)
    return ga, gJ, gr


def ssd_one_warping(fixed: np.ndarray, moving: np.ndarray, lam: float, theta: float,
                    order: int, iters: int) -> float:
    """L = sum (I1(x + w(x)) - I0(x))^2 with w the velocity of one warping."""
    _, J, r = warp_grad_residual(moving, fixed, np.zeros((3,) + fixed.shape))
    w = admm(J, r, lam, theta, order, iters).w
    return ssd(trilinear_periodic(moving, w), fixed)


def ssd_one_warping_grad(fixed: np.ndarray, moving: np.ndarray, lam: float, theta: float,
                         order: int, iters: int):
    """(L, dL/dI1, dL/dlambda) of `ssd_one_warping` (L2 data term), by
    reverse-mode differentiation of the recurrence of `admm`."""
    fixed = np.asarray(fixed, np.float64)
    moving = np.asarray(moving, np.float64)
    dims_xyz = (fixed.shape[2], fixed.shape[1], fixed.shape[0])
    zero_u = np.zeros((3,) + fixed.shape)
    iw, J, r = warp_grad_residual(moving, fixed, zero_u)  # iw == moving exactly at u = 0
    mult = w_step_multiplier(dims_xyz, lam, theta, order)
    kn = laplacian_symbol(dims_xyz) ** order
    dmult = -theta * kn / (theta + lam * kn) ** 2  # d mult / d lambda
    # forward, keeping what the adjoint needs
    zeros = np.zeros_like(J)
    w_hat, b_hat, w_prev, b_prev = zeros, zeros, zeros, zeros
    alpha = 1.0
    tape = []
    for _ in range(iters):
        a = w_hat - b_hat
        v = v_step_l2(a, J, r, theta)
        s = v + b_hat
        w = fourier_solve(s, mult)
        b = s - w
        alpha_next = (1.0 + math.sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0
        g = (alpha - 1.0) / alpha_next
        tape.append((a, s, g))
        w_hat = w + g * (w - w_prev)
        b_hat = b + g * (b - b_prev)
        w_prev, b_prev = w, b
        alpha = alpha_next
    warped = trilinear_periodic(moving, w)
    resid = warped - fixed
    loss = float(np.sum(resid * resid))
    gwarp = 2.0 * resid
    d_moving = trilinear_transpose(gwarp, w)
    # adjoints of w^k and b^k, accumulated as later iterations are reversed
    gw = {iters - 1: gwarp[None] * trilinear_position_gradient(moving, w)}
    gb = {}
    gJ = np.zeros_like(J)
    gr = np.zeros_like(r)
    d_lam = 0.0
    for k in range(iters - 1, -1, -1):
        a, s, _ = tape[k]
        gwk = gw.pop(k, zeros)
        gbk = gb.pop(k, zeros)
        # b = s - w, w = S s
        gw_tot = gwk - gbk
        gs = gbk + fourier_solve(gw_tot, mult)
        d_lam += float(np.sum(gw_tot * fourier_solve(s, dmult)))
        # s = v + b_hat, v = D(a), a = w_hat - b_hat
        ga, gJk, grk = v_step_l2_adjoint(gs, a, J, r, theta)
        gJ += gJk
        gr += grk
        g_what = ga
        g_bhat = gs - ga
        if k >= 1:
            # w_hat^k = w^{k-1} + gamma_{k-1} (w^{k-1} - w^{k-2}) (and b likewise)
            gam = tape[k - 1][2]
            gw[k - 1] = gw.get(k - 1, zeros) + (1.0 + gam) * g_what
            gb[k - 1] = gb.get(k - 1, zeros) + (1.0 + gam) * g_bhat
            if k >= 2:
                gw[k - 2] = gw.get(k - 2, zeros) - gam * g_what
                gb[k - 2] = gb.get(k - 2, zeros) - gam * g_bhat
    # J = grad I1 (central differences: the transpose is minus the same
    # difference), r = I1 - I0, and I1^w = I1 at u = 0
    d_iw = gr.copy()
    for c, ax in enumerate(AXIS_OF_COMPONENT):
        d_iw -= central_diff(gJ[c], ax)
    d_moving += d_iw
    return loss, d_moving, d_lam


# ---------------------------------------------------------------------------
# Three-level pyramid (Sec. 4, first hyper-parameter version)
# ---------------------------------------------------------------------------
# The paper caps the ADMM iterations at 10, 5, 5 and the warpings at 10, 10,
# 5 over three pyramid levels (coarse to fine) and says nothing more.
# Readings: each coarser level halves every dimension by 2x2x2 averaging of
# the images; a level starts from the previous level's displacement carried
# to its grid (coarse voxel i covers fine voxels 2i and 2i + 1, so the
# coarse sample position of fine voxel x is (x - 1/2) / 2, and displacements
# in voxels double); lambda, theta and n are the same at every level.

def downsample2(f: np.ndarray) -> np.ndarray:
    """2x2x2 average of a (nz, ny, nx) volume with even dimensions."""
    nz, ny, nx = f.shape
    return f.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def sample_periodic(f: np.ndarray, px: np.ndarray, py: np.ndarray, pz: np.ndarray) -> np.ndarray:
    """Periodic trilinear value of the (nz, ny, nx) grid function f at the
    points (px, py, pz) (grid coordinates, any shape)."""
    nz, ny, nx = f.shape
    fx, fy, fz = np.floor(px), np.floor(py), np.floor(pz)
    tx, ty, tz = px - fx, py - fy, pz - fz
    x0 = np.mod(fx.astype(np.int64), nx)
    y0 = np.mod(fy.astype(np.int64), ny)
    z0 = np.mod(fz.astype(np.int64), nz)
    x1, y1, z1 = np.mod(x0 + 1, nx), np.mod(y0 + 1, ny), np.mod(z0 + 1, nz)
    return ((1 - tz) * ((1 - ty) * ((1 - tx) * f[z0, y0, x0] + tx * f[z0, y0, x1])
                        + ty * ((1 - tx) * f[z0, y1, x0] + tx * f[z0, y1, x1]))
            + tz * ((1 - ty) * ((1 - tx) * f[z1, y0, x0] + tx * f[z1, y0, x1])
                    + ty * ((1 - tx) * f[z1, y1, x0] + tx * f[z1, y1, x1])))


def upsample2_disp(u: np.ndarray) -> np.ndarray:
    """A coarse displacement (3, nz, ny, nx) carried to the grid twice as
    fine: u_f(x) = 2 u_c((x - 1/2) / 2), periodic trilinear."""
    nz, ny, nx = u.shape[1:]
    zz, yy, xx = np.meshgrid(np.arange(2 * nz), np.arange(2 * ny), np.arange(2 * nx), indexing="ij")
    px, py, pz = (xx - 0.5) / 2.0, (yy - 0.5) / 2.0, (zz - 0.5) / 2.0
    return np.stack([2.0 * sample_periodic(u[c], px, py, pz) for c in range(3)])


def pyramid_register(fixed: np.ndarray, moving: np.ndarray, lam: float, theta: float, order: int,
                     outer=(10, 10, 5), iters=(10, 5, 5), data_term: int = 2,
                     tol_admm: float | None = None, tol_warp: float | None = None) -> RegisterResult:
    """`register` over len(outer) levels, coarsest first, each level starting
    from the previous level's displacement carried to its grid.  With the
    tolerances every level stops its loops by the thresholds of `register`
    (Sec. 4, second hyperparameter version: the pyramid with threshold
    stopping), outer and iters being the caps."""
    levels = len(outer)
    fs = [np.asarray(fixed, np.float64)]
    ms = [np.asarray(moving, np.float64)]
    for _ in range(levels - 1):
        fs.insert(0, downsample2(fs[0]))
        ms.insert(0, downsample2(ms[0]))
    u = None
    res = None
    runs = []
    for lv in range(levels):
        init = None if u is None else upsample2_disp(u)
        res = register(fs[lv], ms[lv], lam, theta, order, outer[lv], iters[lv], data_term=data_term,
                       init_disp=init, tol_admm=tol_admm, tol_warp=tol_warp)
        runs.append(res.iters_run)
        u = res.disp
    res.level_iters = runs
    return res
