"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only *makes inputs*.  It holds none of the registration method's
arithmetic: no trilinear resampling, no ADMM, no Fourier solve and no
scaling-and-squaring.  Smooth random deformations are produced as the time-1
flow of a band-limited stationary velocity field, integrated with classical
RK4 on the continuous field (evaluated between grid points by SciPy's cubic
B-spline interpolation).  Images are evaluated analytically at the deformed
positions (Gaussian blobs, nested ellipsoids).

All generators draw from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed, documented order and return float32 volumes of shape (nz, ny, nx)
(x fastest) and float32 vector fields of shape (3, nz, ny, nx) (component 0
= x), in voxel units.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import ndimage


# ---------------------------------------------------------------------------
# grids and band-limited random fields
# ---------------------------------------------------------------------------
def grid(dims_xyz):
    """Voxel-centre coordinates (x, y, z) as three (nz, ny, nx) float64 arrays."""
    nx, ny, nz = dims_xyz
    zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64),
                             np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    return xx, yy, zz


def band_limited_field(dims_xyz, rng, kmax: int = 4, ncomp: int = 3) -> np.ndarray:
    """Real random field, per component: complex N(0,1) coefficients on every
    integer wavevector with max(|kx|,|ky|,|kz|) <= kmax except DC, real part
    of the inverse DFT.  Normalised so the largest component magnitude is 1."""
    nx, ny, nz = dims_xyz
    out = np.empty((ncomp, nz, ny, nx))
    ks = np.arange(-kmax, kmax + 1)
    for c in range(ncomp):
        spec = np.zeros((nz, ny, nx), dtype=np.complex128)
        coef = rng.standard_normal((len(ks),) * 3) + 1j * rng.standard_normal((len(ks),) * 3)
        for iz, kz in enumerate(ks):
            for iy, ky in enumerate(ks):
                for ix, kx in enumerate(ks):
                    if kx == 0 and ky == 0 and kz == 0:
                        continue
                    spec[kz % nz, ky % ny, kx % nx] += coef[iz, iy, ix]
        out[c] = np.real(np.fft.ifftn(spec))
    return out / np.max(np.abs(out))


def _spline_coeffs(field: np.ndarray) -> np.ndarray:
    return np.stack([ndimage.spline_filter(field[c], order=3, mode="grid-wrap")
                     for c in range(field.shape[0])])


def _eval_field(coeffs: np.ndarray, x, y, z) -> np.ndarray:
    pts = np.stack([z.ravel(), y.ravel(), x.ravel()])
    out = np.stack([ndimage.map_coordinates(coeffs[c], pts, order=3, mode="grid-wrap",
                                            prefilter=False) for c in range(3)])
    return out.reshape((3,) + x.shape)


def flow(coeffs: np.ndarray, scale: float, x0, y0, z0, steps: int = 8) -> np.ndarray:
    """Time-1 flow of dx/dt = scale * v(x) from the given start points, RK4
    with ``steps`` equal steps.  Returns the displacement (3, ...)."""
    h = 1.0 / steps
    x, y, z = x0.copy(), y0.copy(), z0.copy()
    for _ in range(steps):
        k1 = scale * _eval_field(coeffs, x, y, z)
        k2 = scale * _eval_field(coeffs, x + 0.5 * h * k1[0], y + 0.5 * h * k1[1], z + 0.5 * h * k1[2])
        k3 = scale * _eval_field(coeffs, x + 0.5 * h * k2[0], y + 0.5 * h * k2[1], z + 0.5 * h * k2[2])
        k4 = scale * _eval_field(coeffs, x + h * k3[0], y + h * k3[1], z + h * k3[2])
        x = x + h / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        y = y + h / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        z = z + h / 6.0 * (k1[2] + 2 * k2[2] + 2 * k3[2] + k4[2])
    return np.stack([x - x0, y - y0, z - z0])


def smooth_deformation(dims_xyz, rng, max_disp: float, kmax: int = 4,
                       steps: int = 8, sub: int = 4) -> np.ndarray:
    """A random diffeomorphic displacement: the time-1 flow of a band-limited
    velocity, scaled so the largest displacement magnitude over a stride-``sub``
    subsample of start voxels is ``max_disp`` (6 fixed-point rescalings).

    Volumes above 2^18 voxels integrate the flow from every second voxel per
    axis and fill in the rest by periodic cubic B-spline interpolation of
    that (smooth) displacement."""
    vel = band_limited_field(dims_xyz, rng, kmax=kmax)
    coeffs = _spline_coeffs(vel)
    xx, yy, zz = grid(dims_xyz)
    xs, ys, zs = xx[::sub, ::sub, ::sub], yy[::sub, ::sub, ::sub], zz[::sub, ::sub, ::sub]
    scale = max_disp
    for _ in range(6):
        d = flow(coeffs, scale, xs, ys, zs, steps=steps)
        m = float(np.max(np.sqrt(np.sum(d * d, axis=0))))
        scale *= max_disp / m
    nx, ny, nz = dims_xyz
    stride = 2 if nx * ny * nz > (1 << 18) and nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0 else 1
    if stride == 1:
        return flow(coeffs, scale, xx, yy, zz, steps=steps)
    xc, yc, zc = xx[::2, ::2, ::2], yy[::2, ::2, ::2], zz[::2, ::2, ::2]
    coarse = flow(coeffs, scale, xc, yc, zc, steps=steps)
    cc = _spline_coeffs(coarse)
    return _eval_field(cc, xx / 2.0, yy / 2.0, zz / 2.0)


# ---------------------------------------------------------------------------
# Gaussian-blob images
# ---------------------------------------------------------------------------
@dataclass
class Blobs:
    centres: np.ndarray  # (nblob, 3) xyz
    sigmas: np.ndarray
    amps: np.ndarray
    dims_xyz: tuple

    def __call__(self, x, y, z) -> np.ndarray:
        """Sum of isotropic Gaussians with minimum-image periodic distance,
        clipped to [0, 1]; evaluated at arbitrary (x, y, z)."""
        n = self.dims_xyz
        acc = np.zeros(np.shape(x))
        for (cx, cy, cz), s, a in zip(self.centres, self.sigmas, self.amps):
            d2 = 0.0
            for p, c, L in ((x, cx, n[0]), (y, cy, n[1]), (z, cz, n[2])):
                d = np.mod(p - c + L / 2.0, L) - L / 2.0
                d2 = d2 + d * d
            acc += a * np.exp(-d2 / (2.0 * s * s))
        return np.clip(acc, 0.0, 1.0)


def random_blobs(dims_xyz, rng, nblob: int = 6) -> Blobs:
    centres = rng.uniform(0.0, 1.0, size=(nblob, 3)) * np.array(dims_xyz, dtype=np.float64)
    sigmas = rng.uniform(2.0, 5.0, size=nblob)
    amps = rng.uniform(0.3, 1.0, size=nblob)
    return Blobs(centres, sigmas, amps, tuple(dims_xyz))


@dataclass
class Pair:
    fixed: np.ndarray
    moving: np.ndarray
    true_disp: np.ndarray | None = None
    fixed_labels: np.ndarray | None = None
    moving_labels: np.ndarray | None = None


def blob_pair(dims_xyz=(32, 32, 32), seed: int = 0, max_disp: float = 3.0) -> Pair:
    """Gaussian-blob pair: moving = 6 blobs; fixed = the same blobs evaluated
    at x + u(x), u a random smooth diffeomorphic displacement.
    Draw order: blob centres, sigmas, amplitudes, then velocity coefficients."""
    rng = np.random.default_rng(seed)
    blobs = random_blobs(dims_xyz, rng)
    u = smooth_deformation(dims_xyz, rng, max_disp)
    xx, yy, zz = grid(dims_xyz)
    moving = blobs(xx, yy, zz)
    fixed = blobs(xx + u[0], yy + u[1], zz + u[2])
    return Pair(fixed.astype(np.float32), moving.astype(np.float32), u.astype(np.float32))


# ---------------------------------------------------------------------------
# nested-ellipsoid heart phantom (stands in for the 3D cardiac MRI pairs)
# ---------------------------------------------------------------------------
INTENSITY = np.array([0.1, 0.9, 0.4, 0.8])  # background, LV blood, myocardium, RV blood


def phantom_labels(x, y, z, dims_xyz, lv_scale: float = 1.0) -> np.ndarray:
    """Label map of the phantom at arbitrary points (periodic in the volume).

    Geometry for a 128x128x96 volume, scaled per axis by (nx/128, ny/128,
    nz/96): LV centre (56, 64, 48); LV blood semi-axes (11, 11, 22);
    myocardium outer (17, 17, 28); RV blood (12, 20, 24) about (78, 64, 46)
    minus the myocardium's outer ellipsoid.  ``lv_scale`` scales the LV and
    myocardium in-plane (x, y) semi-axes about the LV long (z) axis."""
    nx, ny, nz = dims_xyz
    sx, sy, sz = nx / 128.0, ny / 128.0, nz / 96.0

    def inside(c, ax):
        d2 = 0.0
        for p, cc, a, L in ((x, c[0], ax[0], nx), (y, c[1], ax[1], ny), (z, c[2], ax[2], nz)):
            d = np.mod(p - cc + L / 2.0, L) - L / 2.0
            d2 = d2 + (d / a) ** 2
        return d2 <= 1.0

    lv_c = (56 * sx, 64 * sy, 48 * sz)
    lv = inside(lv_c, (11 * sx * lv_scale, 11 * sy * lv_scale, 22 * sz))
    myo_outer = inside(lv_c, (17 * sx * lv_scale, 17 * sy * lv_scale, 28 * sz))
    rv = inside((78 * sx, 64 * sy, 46 * sz), (12 * sx, 20 * sy, 24 * sz)) & ~myo_outer
    lab = np.zeros(np.shape(x), dtype=np.uint8)
    lab[myo_outer] = 2
    lab[lv] = 1
    lab[rv] = 3
    return lab


def phantom_pair(dims_xyz=(128, 128, 96), seed: int = 1, max_disp: float = 8.0,
                 noise: float = 0.02, contraction: float = 0.9) -> Pair:
    """Cardiac-shaped pair.  moving: the phantom; fixed: the phantom with its
    LV/myocardium contracted in-plane by ``contraction`` and evaluated at
    x + u(x), u a random smooth diffeomorphic displacement (largest magnitude
    ``max_disp`` voxels).  Both get independent N(0, noise^2) noise and are
    clipped to [0, 1].  Draw order: velocity coefficients, moving noise,
    fixed noise."""
    rng = np.random.default_rng(seed)
    u = smooth_deformation(dims_xyz, rng, max_disp)
    xx, yy, zz = grid(dims_xyz)
    lab_m = phantom_labels(xx, yy, zz, dims_xyz)
    lab_f = phantom_labels(xx + u[0], yy + u[1], zz + u[2], dims_xyz, lv_scale=contraction)
    moving = INTENSITY[lab_m] + noise * rng.standard_normal(lab_m.shape)
    fixed = INTENSITY[lab_f] + noise * rng.standard_normal(lab_f.shape)
    return Pair(np.clip(fixed, 0, 1).astype(np.float32), np.clip(moving, 0, 1).astype(np.float32),
                u.astype(np.float32), lab_f, lab_m)


# ---------------------------------------------------------------------------
# generic random inputs for kernel-level parity cases
# ---------------------------------------------------------------------------
def random_volume(dims_xyz, seed: int, smooth_kmax: int | None = None) -> np.ndarray:
    nx, ny, nz = dims_xyz
    rng = np.random.default_rng(seed)
    if smooth_kmax is None:
        return rng.uniform(0.0, 1.0, size=(nz, ny, nx)).astype(np.float32)
    f = band_limited_field(dims_xyz, rng, kmax=smooth_kmax, ncomp=1)[0]
    return (0.5 + 0.5 * f).astype(np.float32)


def random_vector_field(dims_xyz, seed: int, amp: float = 1.0,
                        smooth_kmax: int | None = None) -> np.ndarray:
    nx, ny, nz = dims_xyz
    rng = np.random.default_rng(seed)
    if smooth_kmax is None:
        return (amp * rng.uniform(-1.0, 1.0, size=(3, nz, ny, nx))).astype(np.float32)
    return (amp * band_limited_field(dims_xyz, rng, kmax=smooth_kmax)).astype(np.float32)


# named workloads ------------------------------------------------------------
def bf16_bits(a: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns of float32 values, rounded to nearest, ties to
    even (finite inputs), as uint16."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    """float32 values of bfloat16 bit patterns (exact)."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


WORKLOADS = {
    # 32^3 blob pair, n=2, lambda=0.01, theta=0.1, 5 warpings x 10 iterations
    "blobs32": dict(dims=(32, 32, 32), seed=0, kind="blobs", max_disp=3.0,
                    lam=0.01, theta=0.1, order=2, outer=5, iters=10),
    # 128x128x96 heart phantom, n=2, lambda=0.01, theta=0.1, 10 x 20
    "phantom128x128x96": dict(dims=(128, 128, 96), seed=1, kind="phantom", max_disp=8.0,
                              lam=0.01, theta=0.1, order=2, outer=10, iters=20),
    # 96^3 blob pair for the differentiated warping: one warping of 20
    # iterations, gradients checkpointed every 5 iterations
    "blobs96": dict(dims=(96, 96, 96), seed=3, kind="blobs", max_disp=5.0,
                    lam=0.01, theta=0.1, order=2, outer=1, iters=20, checkpoint=5),
    # 192x192x128 heart phantom (geometry scaled with the volume), images
    # stored as bfloat16 by the precision study; n=3, lambda=0.005, 10 x 30
    "phantom192x192x128": dict(dims=(192, 192, 128), seed=4, kind="phantom", max_disp=8.0,
                               lam=0.005, theta=0.1, order=3, outer=10, iters=30),
}


# Batch of uneven phantom pairs: pair i has seed 1000 + i and a size drawn
# uniformly from BATCH_SIZES by a seed-999 generator; phantom geometry scales
# with the volume, largest displacement 8 voxels.
BATCH_SIZES = ((64, 64, 64), (96, 96, 64), (128, 128, 96))
BATCH_PARAMS = dict(lam=0.01, theta=0.1, order=2, outer=10, iters=20, max_disp=8.0)


def batch_specs(n: int = 32):
    """[(dims_xyz, seed)] of the n pairs of the batch workload."""
    pick = np.random.default_rng(999).integers(0, len(BATCH_SIZES), size=n)
    return [(BATCH_SIZES[int(k)], 1000 + i) for i, k in enumerate(pick)]


def batch_pair(spec) -> tuple:
    """(fixed, moving) of one batch pair (spec from batch_specs)."""
    dims, seed = spec
    p = phantom_pair(dims, seed, BATCH_PARAMS["max_disp"])
    return p.fixed, p.moving


def _cache_dir():
    import os
    d = os.environ.get("NADMM_SYNTH_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "nadmm_synth"))
    try:
        os.makedirs(d, exist_ok=True)
        return d
    except OSError:
        return None


def make_pair(name: str, cache: bool = True) -> Pair:
    """The named workload's image pair (cached as .npz outside the repository)."""
    import os
    w = WORKLOADS[name]
    d = _cache_dir() if cache else None
    path = os.path.join(d, f"{name}_s{w['seed']}_v1.npz") if d else None
    if path and os.path.exists(path):
        z = np.load(path)
        return Pair(**{k: (z[k] if k in z.files else None) for k in Pair.__dataclass_fields__})
    if w["kind"] == "blobs":
        p = blob_pair(w["dims"], w["seed"], w["max_disp"])
    else:
        p = phantom_pair(w["dims"], w["seed"], w["max_disp"])
    if path:
        arrs = {k: v for k, v in p.__dict__.items() if v is not None}
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, **arrs)
        os.replace(tmp, path)
    return p
