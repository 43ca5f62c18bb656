"""Torch-facing wrappers of the C ABI (argument marshalling only).

Volumes are float32 tensors of shape (nz, ny, nx) and vector fields of shape
(3, nz, ny, nx) (component 0 = x), contiguous, on the ROCm device.  Every
function enqueues its work on torch's current stream and returns tensors
whose values are valid in stream order (as with any torch op).
"""
from __future__ import annotations

import ctypes

import numpy as np

import torch

from . import _lib
from ._lib import Dims, Params, Pyramid


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t, name, shape=None, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")


def dims_of(vol_shape) -> Dims:
    nz, ny, nx = vol_shape[-3:]
    return Dims(nx, ny, nz)


def params(lam: float, theta: float, order: int, outer: int = 1, iters: int = 1,
           data_term: int = 2, eps: float = 1e-8) -> Params:
    return Params(float(lam), float(theta), int(order), int(data_term), float(eps), int(outer),
                  int(iters))


def workspace_size(vol_shape) -> int:
    n = ctypes.c_size_t(0)
    _lib.call("nadmm_workspace_size", dims_of(vol_shape), None, ctypes.byref(n))
    return int(n.value)


def workspace(vol_shape, device="cuda") -> torch.Tensor:
    """A workspace tensor usable by every entry point for these dimensions."""
    return torch.empty(workspace_size(vol_shape), dtype=torch.uint8, device=device)


def _ws(vol_shape, ws, device):
    if ws is None:
        ws = workspace(vol_shape, device)
    _check(ws, "workspace", dtype=torch.uint8)
    return ws


def register(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
             outer: int, iters: int, data_term: int = 2, eps: float = 1e-8,
             init_disp: torch.Tensor | None = None, return_velocities: bool = False,
             ws: torch.Tensor | None = None, out: dict | None = None) -> dict:
    """Full registration (Sec. 2 scheme with Sec. 3 ADMM).  Returns a dict with
    'disp' (3, nz, ny, nx), 'warped' (nz, ny, nx) and optionally 'velocities'
    (outer, 3, nz, ny, nx).  ``out`` may supply preallocated output tensors.
    ``fixed`` and ``moving`` are both float32, or both bfloat16 (stored images
    widened to float32 where read; every output is float32)."""
    bf16 = fixed.dtype == torch.bfloat16
    img_dtype = torch.bfloat16 if bf16 else torch.float32
    _check(fixed, "fixed", dtype=img_dtype)
    shp = tuple(fixed.shape)
    _check(moving, "moving", shp, dtype=img_dtype)
    vshp = (3,) + shp
    if init_disp is not None:
        _check(init_disp, "init_disp", vshp)
    out = dict(out or {})
    dev = fixed.device
    disp = out.get("disp")
    if disp is None:
        disp = torch.empty(vshp, dtype=torch.float32, device=dev)
    warped = out.get("warped")
    if warped is None:
        warped = torch.empty(shp, dtype=torch.float32, device=dev)
    vels = out.get("velocities")
    if return_velocities and vels is None:
        vels = torch.empty((outer,) + vshp, dtype=torch.float32, device=dev)
    ws = _ws(shp, ws, dev)
    p = params(lam, theta, order, outer, iters, data_term, eps)
    _lib.call("nadmm_register_bf16" if bf16 else "nadmm_register", dims_of(shp), ctypes.byref(p),
              _ptr(fixed), _ptr(moving),
              _ptr(init_disp), _ptr(disp), _ptr(warped), _ptr(vels) if return_velocities else None,
              _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    res = {"disp": disp, "warped": warped}
    if return_velocities:
        res["velocities"] = vels
    return res


def register_checked(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
                     outer: int, iters: int, finite: bool = True, divergence: bool = True,
                     data_term: int = 2, eps: float = 1e-8, init_disp: torch.Tensor | None = None,
                     ws: torch.Tensor | None = None) -> dict:
    """nadmm_register_checked (synchronous): the registration plus its checks.
    Returns 'disp', 'warped', 'status' (0, NADMM_ERR_NONFINITE = 5 or
    NADMM_ERR_DIVERGED = 6; other errors raise), 'message' and 'diverged'
    (per warping)."""
    _check(fixed, "fixed")
    shp = tuple(fixed.shape)
    _check(moving, "moving", shp)
    vshp = (3,) + shp
    if init_disp is not None:
        _check(init_disp, "init_disp", vshp)
    disp = torch.empty(vshp, dtype=torch.float32, device=fixed.device)
    warped = torch.empty(shp, dtype=torch.float32, device=fixed.device)
    ws = _ws(shp, ws, fixed.device)
    p = params(lam, theta, order, outer, iters, data_term, eps)
    div = (ctypes.c_int32 * max(outer, 1))()
    flags = (_lib.CHECK_FINITE if finite else 0) | (_lib.CHECK_DIVERGENCE if divergence else 0)
    st = _lib.load().nadmm_register_checked(dims_of(shp), ctypes.byref(p), ctypes.c_uint32(flags), _ptr(fixed),
                                            _ptr(moving), _ptr(init_disp), _ptr(disp), _ptr(warped), div,
                                            _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    msg = _lib.load().nadmm_last_error().decode(errors="replace") if st else ""
    if st not in (0, 5, 6):
        _lib.check("nadmm_register_checked", st)
    return {"disp": disp, "warped": warped, "status": int(st), "message": msg, "diverged": list(div)[:outer]}


def register_threshold(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
                       outer: int, iters: int, tol_admm: float, tol_warp: float, data_term: int = 2,
                       eps: float = 1e-8, ws: torch.Tensor | None = None) -> dict:
    """Registration with threshold stopping (nadmm_register_threshold): the
    ADMM loop stops once |s^k - s^{k-1}| <= tol_admm |s^k|, the warping loop
    once |u_c - u_{c-1}| <= tol_warp |u_c| (negative: no check); ``outer``
    and ``iters`` stay the caps.  Synchronous.  Returns 'disp', 'warped',
    'iters_run' (per warping run), 'outer_run', 'admm_change' (per warping
    run, the changes measured: not at an iteration that ends at the cap) and
    'warp_change' (likewise, for the warpings from the second on)."""
    _check(fixed, "fixed")
    shp = tuple(fixed.shape)
    _check(moving, "moving", shp)
    dev = fixed.device
    disp = torch.empty((3,) + shp, dtype=torch.float32, device=dev)
    warped = torch.empty(shp, dtype=torch.float32, device=dev)
    ws = _ws(shp, ws, dev)
    p = params(lam, theta, order, outer, iters, data_term, eps)
    runs = (ctypes.c_int32 * max(outer, 1))()
    n_run = ctypes.c_int32(0)
    achg = (ctypes.c_double * max(outer * (iters - 1), 1))()
    wchg = (ctypes.c_double * max(outer - 1, 1))()
    _lib.call("nadmm_register_threshold", dims_of(shp), ctypes.byref(p), ctypes.c_double(tol_admm),
              ctypes.c_double(tol_warp), _ptr(fixed), _ptr(moving), _ptr(disp), _ptr(warped), runs,
              ctypes.byref(n_run), achg, wchg, _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    oc = n_run.value
    its = [runs[c] for c in range(oc)]
    admm_change = [[x for x in (achg[c * (iters - 1) + k] for k in range(its[c] - 1)) if x == x]
                   for c in range(oc)]  # NaN: not measured
    return {"disp": disp, "warped": warped, "iters_run": its, "outer_run": oc,
            "admm_change": admm_change,
            "warp_change": [x for x in (wchg[c] for c in range(max(oc - 1, 0))) if x == x]}


def workspace_batch(vol_shape, batch: int, device="cuda") -> torch.Tensor:
    n = ctypes.c_size_t(0)
    _lib.call("nadmm_workspace_size_batch", dims_of(vol_shape), ctypes.c_int32(batch), ctypes.byref(n))
    return torch.empty(int(n.value), dtype=torch.uint8, device=device)


def register_batch(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
                   outer: int, iters: int, data_term: int = 2, eps: float = 1e-8,
                   init_disp: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                   out: dict | None = None) -> dict:
    """``batch`` pairs of one size in one call: fixed, moving (batch, nz, ny, nx)
    float32; returns 'disp' (batch, 3, nz, ny, nx) and 'warped' (batch, nz,
    ny, nx).  Bit-identical to registering the pairs one by one."""
    _check(fixed, "fixed")
    shp = tuple(fixed.shape)
    if len(shp) != 4:
        raise ValueError("fixed must have shape (batch, nz, ny, nx)")
    _check(moving, "moving", shp)
    b, vol = shp[0], shp[1:]
    vshp = (b, 3) + vol
    if init_disp is not None:
        _check(init_disp, "init_disp", vshp)
    out = dict(out or {})
    disp = out.get("disp")
    if disp is None:
        disp = torch.empty(vshp, dtype=torch.float32, device=fixed.device)
    warped = out.get("warped")
    if warped is None:
        warped = torch.empty(shp, dtype=torch.float32, device=fixed.device)
    if ws is None:
        ws = workspace_batch(vol, b, fixed.device)
    _check(ws, "workspace", dtype=torch.uint8)
    p = params(lam, theta, order, outer, iters, data_term, eps)
    _lib.call("nadmm_register_batch", dims_of(vol), ctypes.c_int32(b), ctypes.byref(p), _ptr(fixed),
              _ptr(moving), _ptr(init_disp), _ptr(disp), _ptr(warped), _ptr(ws),
              ctypes.c_size_t(ws.numel()), _stream())
    return {"disp": disp, "warped": warped}


def _dims_array(shapes):
    arr = (Dims * len(shapes))()
    for i, shp in enumerate(shapes):
        arr[i] = dims_of(shp)
    return arr


def workspace_mixed(shapes, device="cuda") -> torch.Tensor:
    """Workspace of register_mixed for pairs of the given (nz, ny, nx) shapes
    (any order: the size is that of the grouped order)."""
    n = ctypes.c_size_t(0)
    shapes = [tuple(shapes[i]) for i in mixed_order(shapes)]
    _lib.call("nadmm_workspace_size_mixed", ctypes.c_int32(len(shapes)), _dims_array(shapes), ctypes.byref(n))
    return torch.empty(int(n.value), dtype=torch.uint8, device=device)


def mixed_order(shapes) -> list:
    """Pair order that puts pairs of one size together (sizes in order of
    first appearance, pairs of a size in their given order)."""
    first = {}
    for i, shp in enumerate(shapes):
        first.setdefault(tuple(shp), i)
    return sorted(range(len(shapes)), key=lambda i: (first[tuple(shapes[i])], i))


def register_mixed(fixed: list, moving: list, lam: float, theta: float, order: int, outer: int, iters: int,
                   data_term: int = 2, eps: float = 1e-8, ws: torch.Tensor | None = None,
                   packed: tuple | None = None) -> dict:
    """Pairs of several sizes in one call, one launch per phase over all of
    them (nadmm_register_mixed).  fixed, moving: lists of float32 (nz, ny, nx)
    tensors in any order (they are grouped by size for the call).  Returns
    'disp' and 'warped' lists in the given order (views into one buffer
    each) and 'packed' = (fixed, moving, disp, warped) flat buffers in the
    grouped order, which a later call may pass back as `packed` to reuse."""
    shapes = [tuple(f.shape) for f in fixed]
    if len(moving) != len(fixed):
        raise ValueError("fixed and moving must have the same number of pairs")
    for f, m in zip(fixed, moving):
        _check(f, "fixed")
        _check(m, "moving", tuple(f.shape))
    dev = fixed[0].device
    perm = mixed_order(shapes)
    gshapes = [shapes[i] for i in perm]
    sizes = [int(np.prod(shp)) for shp in gshapes]
    if packed is None:
        f_flat = torch.cat([fixed[i].reshape(-1) for i in perm])
        m_flat = torch.cat([moving[i].reshape(-1) for i in perm])
        d_flat = torch.empty(3 * sum(sizes), dtype=torch.float32, device=dev)
        w_flat = torch.empty(sum(sizes), dtype=torch.float32, device=dev)
    else:
        f_flat, m_flat, d_flat, w_flat = packed
    if ws is None:
        ws = workspace_mixed(gshapes, dev)
    _check(ws, "workspace", dtype=torch.uint8)
    p = params(lam, theta, order, outer, iters, data_term, eps)
    _lib.call("nadmm_register_mixed", ctypes.c_int32(len(gshapes)), _dims_array(gshapes), ctypes.byref(p),
              _ptr(f_flat), _ptr(m_flat), _ptr(d_flat), _ptr(w_flat), _ptr(ws), ctypes.c_size_t(ws.numel()),
              _stream())
    disp, warped = [None] * len(shapes), [None] * len(shapes)
    o = 0
    for i, shp, n in zip(perm, gshapes, sizes):
        disp[i] = d_flat[3 * o:3 * (o + n)].view((3,) + shp)
        warped[i] = w_flat[o:o + n].view(shp)
        o += n
    return {"disp": disp, "warped": warped, "packed": (f_flat, m_flat, d_flat, w_flat)}


def workspace_grad(vol_shape, lam: float, theta: float, order: int, iters: int, checkpoint: int,
                   device="cuda") -> torch.Tensor:
    n = ctypes.c_size_t(0)
    p = params(lam, theta, order, 1, iters)
    _lib.call("nadmm_workspace_size_grad", dims_of(vol_shape), ctypes.byref(p), ctypes.c_int32(checkpoint),
              ctypes.byref(n))
    return torch.empty(int(n.value), dtype=torch.uint8, device=device)


def ssd_grad(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
             iters: int, checkpoint: int = 5, ws: torch.Tensor | None = None, loss_only: bool = False):
    """Loss, dL/dmoving and dL/dlambda of one warping's image match
    L = sum (moving(x + w(x)) - fixed(x))^2 (see nadmm_ssd_grad).  Returns
    (loss, d_moving, d_lambda) with loss and d_lambda float64 0-d tensors
    (loss_only: (loss, None, None), no reverse pass)."""
    _check(fixed, "fixed")
    shp = tuple(fixed.shape)
    _check(moving, "moving", shp)
    if ws is None:
        ws = workspace_grad(shp, lam, theta, order, iters, checkpoint, fixed.device)
    _check(ws, "workspace", dtype=torch.uint8)
    loss = torch.empty((), dtype=torch.float64, device=fixed.device)
    dlam = None if loss_only else torch.empty((), dtype=torch.float64, device=fixed.device)
    dmov = None if loss_only else torch.empty_like(moving)
    p = params(lam, theta, order, 1, iters)
    _lib.call("nadmm_ssd_grad", dims_of(shp), ctypes.byref(p), ctypes.c_int32(checkpoint), _ptr(fixed),
              _ptr(moving), _ptr(loss), _ptr(dmov), _ptr(dlam), _ptr(ws), ctypes.c_size_t(ws.numel()),
              _stream())
    return loss, dmov, dlam


def pyramid(outer=(10, 10, 5), iters=(10, 5, 5)) -> Pyramid:
    if len(outer) != len(iters) or not 1 <= len(outer) <= 4:
        raise ValueError("outer and iters need one entry per level (1 to 4 levels)")
    py = Pyramid()
    py.levels = len(outer)
    for i, (o, k) in enumerate(zip(outer, iters)):
        py.outer[i] = int(o)
        py.iters[i] = int(k)
    return py


def workspace_pyramid(vol_shape, outer=(10, 10, 5), iters=(10, 5, 5), device="cuda") -> torch.Tensor:
    """Workspace of register_pyramid for this schedule."""
    py = pyramid(outer, iters)
    n = ctypes.c_size_t(0)
    _lib.call("nadmm_workspace_size_pyramid", dims_of(vol_shape), ctypes.byref(py), ctypes.byref(n))
    return torch.empty(int(n.value), dtype=torch.uint8, device=device)


def register_pyramid(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
                     outer=(10, 10, 5), iters=(10, 5, 5), data_term: int = 2, eps: float = 1e-8,
                     ws: torch.Tensor | None = None) -> dict:
    """Multi-resolution registration, coarsest level first (see
    nadmm_register_pyramid); the defaults are the paper's caps of its first
    hyper-parameter version.  Returns 'disp' and 'warped' at full size."""
    _check(fixed, "fixed")
    shp = tuple(fixed.shape)
    _check(moving, "moving", shp)
    py = pyramid(outer, iters)
    if ws is None:
        ws = workspace_pyramid(shp, outer, iters, fixed.device)
    _check(ws, "workspace", dtype=torch.uint8)
    disp = torch.empty((3,) + shp, dtype=torch.float32, device=fixed.device)
    warped = torch.empty(shp, dtype=torch.float32, device=fixed.device)
    p = params(lam, theta, order, 1, 1, data_term, eps)
    _lib.call("nadmm_register_pyramid", dims_of(shp), ctypes.byref(p), ctypes.byref(py), _ptr(fixed),
              _ptr(moving), _ptr(disp), _ptr(warped), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    return {"disp": disp, "warped": warped}


def register_pyramid_threshold(fixed: torch.Tensor, moving: torch.Tensor, lam: float, theta: float, order: int,
                               outer, iters, tol_admm: float, tol_warp: float, data_term: int = 2,
                               eps: float = 1e-8, ws: torch.Tensor | None = None) -> dict:
    """The pyramid with threshold stopping at every level
    (nadmm_register_pyramid_threshold; ``outer`` / ``iters`` per level are
    the caps).  Synchronous.  Returns 'disp', 'warped', 'level_iters' (per
    level, the ADMM iterations of each warping run) and 'outer_run'."""
    _check(fixed, "fixed")
    shp = tuple(fixed.shape)
    _check(moving, "moving", shp)
    py = pyramid(outer, iters)
    if ws is None:
        ws = workspace_pyramid(shp, outer, iters, fixed.device)
    _check(ws, "workspace", dtype=torch.uint8)
    disp = torch.empty((3,) + shp, dtype=torch.float32, device=fixed.device)
    warped = torch.empty(shp, dtype=torch.float32, device=fixed.device)
    p = params(lam, theta, order, 1, 1, data_term, eps)
    runs = (ctypes.c_int32 * max(sum(outer), 1))()
    oruns = (ctypes.c_int32 * len(outer))()
    _lib.call("nadmm_register_pyramid_threshold", dims_of(shp), ctypes.byref(p), ctypes.byref(py),
              ctypes.c_double(tol_admm), ctypes.c_double(tol_warp), _ptr(fixed), _ptr(moving), _ptr(disp),
              _ptr(warped), runs, oruns, _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    level_iters, at = [], 0
    for lv, n in enumerate(outer):
        level_iters.append([runs[at + c] for c in range(oruns[lv])])
        at += n
    return {"disp": disp, "warped": warped, "level_iters": level_iters, "outer_run": list(oruns)}


def autotune(vol_shape, lam: float, theta: float, order: int, batch: int = 1,
             ws: torch.Tensor | None = None, device="cuda") -> int:
    """Pick and keep the fastest x-line tile for these sizes (see
    nadmm_autotune); returns the rows per workgroup chosen."""
    if ws is None:
        ws = workspace_batch(vol_shape, batch, device)
    rows = ctypes.c_int32(0)
    p = params(lam, theta, order)
    _lib.call("nadmm_autotune", dims_of(vol_shape), ctypes.c_int32(batch), ctypes.byref(p), _ptr(ws),
              ctypes.c_size_t(ws.numel()), _stream(), ctypes.byref(rows))
    return int(rows.value)


def tuned_shapes(vol_shape) -> dict:
    """Launch shapes in use for these sizes (nadmm_tuned_shapes)."""
    out = (ctypes.c_int32 * 3)()
    _lib.call("nadmm_tuned_shapes", dims_of(vol_shape), out)
    return {"xline_rows": out[0], "compose_rows": out[1], "plane_threads": out[2]}


def set_shapes(vol_shape, xline_rows: int = 0, compose_rows: int = 0, plane_threads: int = 0) -> None:
    """Pins the launch shapes for these sizes without timing (nadmm_set_shapes;
    0 restores a shape's default)."""
    arr = (ctypes.c_int32 * 3)(xline_rows, compose_rows, plane_threads)
    _lib.call("nadmm_set_shapes", dims_of(vol_shape), arr)


def admm(J: torch.Tensor, r: torch.Tensor, lam: float, theta: float, order: int, iters: int,
         data_term: int = 2, eps: float = 1e-8, ws: torch.Tensor | None = None):
    """``iters`` ADMM iterations from zero for a given J, r.  Returns (w, b, v)."""
    _check(r, "r")
    shp = tuple(r.shape)
    _check(J, "J", (3,) + shp)
    w, b, v = (torch.empty_like(J) for _ in range(3))
    ws = _ws(shp, ws, r.device)
    p = params(lam, theta, order, 1, iters, data_term, eps)
    _lib.call("nadmm_admm", dims_of(shp), ctypes.byref(p), _ptr(J), _ptr(r), _ptr(w), _ptr(b),
              _ptr(v), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    return w, b, v


def fourier_solve(s: torch.Tensor, lam: float, theta: float, order: int,
                  ws: torch.Tensor | None = None) -> torch.Tensor:
    """w = F^-1[theta F(s) / (theta + lam K^order)] per component."""
    _check(s, "s")
    shp = tuple(s.shape[1:])
    _check(s, "s", (3,) + shp)
    w = torch.empty_like(s)
    ws = _ws(shp, ws, s.device)
    p = params(lam, theta, order)
    _lib.call("nadmm_fourier_solve", dims_of(shp), ctypes.byref(p), _ptr(s), _ptr(w), _ptr(ws),
              ctypes.c_size_t(ws.numel()), _stream())
    return w


def warp(img: torch.Tensor, disp: torch.Tensor, ref: torch.Tensor | None = None,
         grad: bool = False):
    """Returns (warped, grad or None, resid or None)."""
    _check(img, "img")
    shp = tuple(img.shape)
    _check(disp, "disp", (3,) + shp)
    if ref is not None:
        _check(ref, "ref", shp)
    out = torch.empty_like(img)
    g = torch.empty_like(disp) if grad else None
    rs = torch.empty_like(img) if ref is not None else None
    _lib.call("nadmm_warp", dims_of(shp), _ptr(img), _ptr(disp), _ptr(ref), _ptr(out), _ptr(g),
              _ptr(rs), _stream())
    return out, g, rs


def compose(u: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """Displacement of (Id + u) o (Id + v): v(x) + u(x + v(x))."""
    _check(u, "u")
    _check(v, "v", tuple(u.shape))
    out = torch.empty_like(u)
    _lib.call("nadmm_compose", dims_of(u.shape), _ptr(u), _ptr(v), _ptr(out), _stream())
    return out


def expmap(vel: torch.Tensor, steps: int, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Scaling and squaring with ``steps`` squarings."""
    _check(vel, "vel")
    shp = tuple(vel.shape[1:])
    out = torch.empty_like(vel)
    ws = _ws(shp, ws, vel.device)
    _lib.call("nadmm_expmap", dims_of(shp), _ptr(vel), ctypes.c_int32(steps), _ptr(out), _ptr(ws),
              ctypes.c_size_t(ws.numel()), _stream())
    return out


def jacobian(disp: torch.Tensor, want_det: bool = False, ws: torch.Tensor | None = None):
    """Returns (stats, n_nonpos, det): stats = float64 [min, max, mean] of
    det(I + D disp), n_nonpos = int64 [count of det <= 0], det optional."""
    _check(disp, "disp")
    shp = tuple(disp.shape[1:])
    det = torch.empty(shp, dtype=torch.float32, device=disp.device) if want_det else None
    stats = torch.empty(3, dtype=torch.float64, device=disp.device)
    nneg = torch.empty(1, dtype=torch.int64, device=disp.device)
    ws = _ws(shp, ws, disp.device)
    _lib.call("nadmm_jacobian", dims_of(shp), _ptr(disp), _ptr(det), _ptr(stats), _ptr(nneg),
              _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    return stats, nneg, det


def jacobian_noalloc(disp: torch.Tensor, want_det: bool = False):
    """jacobian() through nadmm_jacobian_noalloc: no workspace, the
    reduction's partials in the library's own device array."""
    _check(disp, "disp")
    shp = tuple(disp.shape[1:])
    det = torch.empty(shp, dtype=torch.float32, device=disp.device) if want_det else None
    stats = torch.empty(3, dtype=torch.float64, device=disp.device)
    nneg = torch.empty(1, dtype=torch.int64, device=disp.device)
    _lib.call("nadmm_jacobian_noalloc", dims_of(shp), _ptr(disp), _ptr(det), _ptr(stats), _ptr(nneg),
              _stream())
    return stats, nneg, det


def count_nonfinite(field: torch.Tensor) -> torch.Tensor:
    """Device int64 [1]: number of NaN or infinite entries of a scalar volume
    (nz, ny, nx) or of stacked volumes (C, nz, ny, nx)."""
    _check(field, "field")
    if field.dim() not in (3, 4):
        raise ValueError("field must be (nz, ny, nx) or (C, nz, ny, nx)")
    count = 1 if field.dim() == 3 else field.shape[0]
    out = torch.empty(1, dtype=torch.int64, device=field.device)
    _lib.call("nadmm_count_nonfinite", dims_of(field.shape), _ptr(field), ctypes.c_int32(count),
              _ptr(out), _stream())
    return out


REPLAY_KINDS = {"pass_a_fwd_x": 0, "pass_b_yz_solve": 1, "pass_ca_iter": 2, "admm_iteration": 3}


def profile_replay(vol_shape, kind: str, reps: int, lam: float, theta: float, order: int,
                   ws: torch.Tensor, data_term: int = 2, eps: float = 1e-8) -> float:
    """Mean milliseconds of one iteration kernel replayed ``reps`` times back to
    back on the state a preceding register() call left in ``ws``."""
    p = params(lam, theta, order, 1, 2, data_term, eps)
    ms = ctypes.c_double(0.0)
    _lib.call("nadmm_profile_replay", dims_of(vol_shape), ctypes.byref(p), ctypes.c_int32(REPLAY_KINDS[kind]),
              ctypes.c_int32(reps), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(), ctypes.byref(ms))
    return float(ms.value)
