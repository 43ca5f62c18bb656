"""The oracle's registration (Sec. 2 scheme, Sec. 3 Eq. (5) and (6)) with
every array held in float32: the same steps in the same order as
oracle.register, NumPy float32 arithmetic and scipy.fft in float32.

Test infrastructure, not an oracle: it measures how far float32 arithmetic
alone, with no GPU involved, moves a registration from the FP64 oracle.  At
an ill-conditioned workload (one whose deformation folds) that distance sets
the scale of the agreement any float32 implementation can reach near the
folds; make_golden.py records it beside the FP64 samples.
"""
import numpy as np
import scipy.fft as sfft

import oracle as O

F32 = np.float32


def _central_diff(f, axis):
    return (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)) * F32(0.5)


def _gradient(f):
    return np.stack([_central_diff(f, ax) for ax in O.AXIS_OF_COMPONENT])


def _trilinear(f, disp):
    """Periodic trilinear sampling at x + disp(x) with the cell split exactly
    (integer part x + floor(disp), fraction disp - floor(disp)) in float32."""
    nz, ny, nx = disp.shape[1:]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    fl = [np.floor(disp[c]) for c in range(3)]
    tx, ty, tz = (disp[c] - fl[c] for c in range(3))
    ix0 = np.mod(xx + fl[0].astype(np.int64), nx)
    iy0 = np.mod(yy + fl[1].astype(np.int64), ny)
    iz0 = np.mod(zz + fl[2].astype(np.int64), nz)
    ix1, iy1, iz1 = np.mod(ix0 + 1, nx), np.mod(iy0 + 1, ny), np.mod(iz0 + 1, nz)

    def lerp(a, b, t):
        return a + t * (b - a)

    def one(g):
        c00 = lerp(g[iz0, iy0, ix0], g[iz0, iy0, ix1], tx)
        c10 = lerp(g[iz0, iy1, ix0], g[iz0, iy1, ix1], tx)
        c01 = lerp(g[iz1, iy0, ix0], g[iz1, iy0, ix1], tx)
        c11 = lerp(g[iz1, iy1, ix0], g[iz1, iy1, ix1], tx)
        return lerp(lerp(c00, c10, ty), lerp(c01, c11, ty), tz)

    return one(f) if f.ndim == 3 else np.stack([one(f[c]) for c in range(f.shape[0])])


def register_fp32(fixed, moving, lam, theta, order, outer, iters):
    """oracle.register (L2 data term, fixed counts, from u = 0) in float32.
    Returns (disp, warped), both float32."""
    fixed, moving = np.asarray(fixed, F32), np.asarray(moving, F32)
    nz, ny, nx = fixed.shape
    mult = O.w_step_multiplier((nx, ny, nz), lam, theta, order).astype(F32)
    gam = O.nesterov_gammas(iters).astype(F32)
    th = F32(theta)
    u = np.zeros((3,) + fixed.shape, F32)
    for _ in range(outer):
        iw = _trilinear(moving, u)
        J, r = _gradient(iw), iw - fixed
        jj = np.sum(J * J, axis=0)
        zero = np.zeros_like(J)
        w_hat = b_hat = w_prev = b_prev = zero
        for k in range(iters):
            a = w_hat - b_hat
            v = a - J * ((np.sum(J * a, axis=0) + r) / (th + jj))[None]
            s = v + b_hat
            w = np.stack([sfft.irfftn(mult * sfft.rfftn(s[c], axes=(0, 1, 2)), s=s.shape[1:], axes=(0, 1, 2))
                          for c in range(3)]).astype(F32)
            b = b_hat + v - w
            w_hat = w + gam[k] * (w - w_prev)
            b_hat = b + gam[k] * (b - b_prev)
            w_prev, b_prev = w, b
        u = w + _trilinear(u, w)
    return u, _trilinear(moving, u)
