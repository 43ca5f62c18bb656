"""Guard bands: no kernel writes outside the buffers it is given.

Every input, output and workspace of the entry points below is placed in
the middle of a larger device allocation whose 64 KB head and tail are
filled with a sentinel byte; after the call (through the C ABI) the head and
tail must hold the sentinel, the inputs must be unchanged, and every output
must equal that of the same call on plain buffers bit for bit.  Sizes: a
half-plane grid (16 x 192 x 96: y-z planes of 18432 points, transformed
as two half planes after a radix-2 y step in the x-line passes), a ragged
one-plane grid (24 x 18 x 12) and a
batch of 3 pairs; the pyramid runs three levels down from 32 x 192 x 96.
"""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = 64 * 1024
SENT = 0xA5
DIMS = [(16, 192, 96), (24, 18, 12)]
LAM, THETA, ORDER = 0.01, 0.1, 2


@pytest.fixture(scope="module")
def lib():
    from paper_2109_12688_amd import _lib
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _lib.load()
    return _lib


class Guarded:
    """`nbytes` of device memory between two sentinel-filled guard bands."""

    def __init__(self, nbytes, content=None):
        self.n = int(nbytes)
        self.buf = torch.full((self.n + 2 * G,), SENT, dtype=torch.uint8, device="cuda")
        if content is not None:
            src = content.contiguous().view(torch.uint8).reshape(-1)
            assert src.numel() == self.n
            self.buf[G:G + self.n].copy_(src)
        self.before = None if content is None else self.inner().clone()

    def inner(self):
        return self.buf[G:G + self.n]

    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr() + G)

    def check(self, name):
        torch.cuda.synchronize()
        head, tail = self.buf[:G], self.buf[G + self.n:]
        assert bool((head == SENT).all()), f"{name}: write before the buffer"
        assert bool((tail == SENT).all()), f"{name}: write after the buffer"
        if self.before is not None:
            assert torch.equal(self.inner(), self.before), f"{name}: input modified"


class Plain:
    def __init__(self, nbytes, content=None):
        self.n = int(nbytes)
        self.t = torch.zeros(self.n, dtype=torch.uint8, device="cuda")
        if content is not None:
            self.t.copy_(content.contiguous().view(torch.uint8).reshape(-1))

    def inner(self):
        return self.t

    def ptr(self):
        return ctypes.c_void_p(self.t.data_ptr())

    def check(self, name):
        pass


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dims(lib, d):
    return lib.Dims(*d)


def _params(lib, outer, iters, data_term=2):
    return lib.Params(LAM, THETA, ORDER, data_term, 1e-8, outer, iters)


def _ws_bytes(lib, fn, *args):
    n = ctypes.c_size_t(0)
    lib.call(fn, *args, ctypes.byref(n))
    return n.value


def _images(d, seed, batch=1):
    vols = [synth.random_volume(d, seed=seed + 2 * i, smooth_kmax=3) for i in range(2 * batch)]
    f = torch.from_numpy(np.stack(vols[0::2]).astype(np.float32)).cuda()
    m = torch.from_numpy(np.stack(vols[1::2]).astype(np.float32)).cuda()
    return f, m


def _run_both(call, specs):
    """Runs call(bufs) on guarded and on plain buffers; checks the guards and
    inputs and compares every buffer's final bytes (outputs bit for bit; the
    workspace, key 'ws', is scratch and not compared)."""
    res = {}
    for kind in (Guarded, Plain):
        bufs = {k: kind(n, c) for k, (n, c) in specs.items()}
        call(bufs)
        torch.cuda.synchronize()
        for k, b in bufs.items():
            b.check(k)
        res[kind] = {k: b.inner().clone() for k, b in bufs.items()}
    for k in specs:
        if k != "ws":
            assert torch.equal(res[Guarded][k], res[Plain][k]), f"{k} differs from the plain call"


@pytest.mark.parametrize("d", DIMS)
def test_guard_register_and_bf16(lib, d):
    V = int(np.prod(d))
    f, m = _images(d, 300)
    init = torch.from_numpy(synth.random_vector_field(d, seed=301, amp=0.5, smooth_kmax=2)).cuda()
    outer, iters = 2, 3
    wsb = _ws_bytes(lib, "nadmm_workspace_size", _dims(lib, d), None)
    specs = {"fixed": (4 * V, f), "moving": (4 * V, m), "init": (12 * V, init), "disp": (12 * V, None),
             "warped": (4 * V, None), "vel": (12 * V * outer, None), "ws": (wsb, None)}
    p = _params(lib, outer, iters)

    def call(b):
        lib.call("nadmm_register", _dims(lib, d), ctypes.byref(p), b["fixed"].ptr(), b["moving"].ptr(),
                 b["init"].ptr(), b["disp"].ptr(), b["warped"].ptr(), b["vel"].ptr(), b["ws"].ptr(),
                 ctypes.c_size_t(wsb), _stream())
    _run_both(call, specs)
    fb, mb = f.to(torch.bfloat16), m.to(torch.bfloat16)
    specs.update({"fixed": (2 * V, fb), "moving": (2 * V, mb)})

    def call16(b):
        lib.call("nadmm_register_bf16", _dims(lib, d), ctypes.byref(p), b["fixed"].ptr(), b["moving"].ptr(),
                 b["init"].ptr(), b["disp"].ptr(), b["warped"].ptr(), b["vel"].ptr(), b["ws"].ptr(),
                 ctypes.c_size_t(wsb), _stream())
    _run_both(call16, specs)


@pytest.mark.parametrize("d", DIMS)
def test_guard_batch_of_three(lib, d):
    V, B = int(np.prod(d)), 3
    f, m = _images(d, 310, batch=B)
    wsb = _ws_bytes(lib, "nadmm_workspace_size_batch", _dims(lib, d), ctypes.c_int32(B))
    specs = {"fixed": (4 * V * B, f), "moving": (4 * V * B, m), "disp": (12 * V * B, None),
             "warped": (4 * V * B, None), "ws": (wsb, None)}
    p = _params(lib, 2, 3)

    def call(b):
        lib.call("nadmm_register_batch", _dims(lib, d), ctypes.c_int32(B), ctypes.byref(p), b["fixed"].ptr(),
                 b["moving"].ptr(), None, b["disp"].ptr(), b["warped"].ptr(), b["ws"].ptr(),
                 ctypes.c_size_t(wsb), _stream())
    _run_both(call, specs)


def test_guard_pyramid(lib):
    d = (32, 192, 96)
    V = int(np.prod(d))
    f, m = _images(d, 320)
    py = lib.Pyramid(3, (ctypes.c_int32 * 4)(2, 2, 1, 0), (ctypes.c_int32 * 4)(2, 2, 2, 0))
    wsb = _ws_bytes(lib, "nadmm_workspace_size_pyramid", _dims(lib, d), ctypes.byref(py))
    specs = {"fixed": (4 * V, f), "moving": (4 * V, m), "disp": (12 * V, None), "warped": (4 * V, None),
             "ws": (wsb, None)}
    p = _params(lib, 1, 1)

    def call(b):
        lib.call("nadmm_register_pyramid", _dims(lib, d), ctypes.byref(p), ctypes.byref(py), b["fixed"].ptr(),
                 b["moving"].ptr(), b["disp"].ptr(), b["warped"].ptr(), b["ws"].ptr(), ctypes.c_size_t(wsb),
                 _stream())
    _run_both(call, specs)


@pytest.mark.parametrize("d", DIMS)
def test_guard_threshold_and_gradient(lib, d):
    V = int(np.prod(d))
    f, m = _images(d, 330)
    wsb = _ws_bytes(lib, "nadmm_workspace_size", _dims(lib, d), None)
    outer, iters = 3, 4
    specs = {"fixed": (4 * V, f), "moving": (4 * V, m), "disp": (12 * V, None), "warped": (4 * V, None),
             "ws": (wsb, None)}
    p = _params(lib, outer, iters)

    def call(b):
        runs = (ctypes.c_int32 * outer)()
        n_run = ctypes.c_int32(0)
        achg = (ctypes.c_double * (outer * (iters - 1)))()
        wchg = (ctypes.c_double * (outer - 1))()
        lib.call("nadmm_register_threshold", _dims(lib, d), ctypes.byref(p), ctypes.c_double(1e-3),
                 ctypes.c_double(0.0), b["fixed"].ptr(), b["moving"].ptr(), b["disp"].ptr(), b["warped"].ptr(),
                 runs, ctypes.byref(n_run), achg, wchg, b["ws"].ptr(), ctypes.c_size_t(wsb), _stream())
    _run_both(call, specs)
    ck = 2
    wsg = _ws_bytes(lib, "nadmm_workspace_size_grad", _dims(lib, d), ctypes.byref(p), ctypes.c_int32(ck))
    specs = {"fixed": (4 * V, f), "moving": (4 * V, m), "loss": (8, None), "dmov": (4 * V, None),
             "dlam": (8, None), "ws": (wsg, None)}

    def call_grad(b):
        lib.call("nadmm_ssd_grad", _dims(lib, d), ctypes.byref(p), ctypes.c_int32(ck), b["fixed"].ptr(),
                 b["moving"].ptr(), b["loss"].ptr(), b["dmov"].ptr(), b["dlam"].ptr(), b["ws"].ptr(),
                 ctypes.c_size_t(wsg), _stream())
    # d_moving is a scatter-add with float atomics: compare the guards and
    # inputs only, the values to a tolerance
    for kind in (Guarded, Plain):
        bufs = {k: kind(n, c) for k, (n, c) in specs.items()}
        call_grad(bufs)
        torch.cuda.synchronize()
        for k, b in bufs.items():
            b.check(k)
        if kind is Guarded:
            g = bufs["dmov"].inner().view(torch.float32).clone()
        else:
            h = bufs["dmov"].inner().view(torch.float32)
            assert torch.allclose(g, h, rtol=1e-5, atol=1e-6 * float(h.abs().max()))


@pytest.mark.parametrize("d", DIMS)
def test_guard_single_steps(lib, d):
    V = int(np.prod(d))
    f, m = _images(d, 340)
    u = torch.from_numpy(synth.random_vector_field(d, seed=341, amp=2.0, smooth_kmax=2)).cuda()
    v = torch.from_numpy(synth.random_vector_field(d, seed=342, amp=1.0, smooth_kmax=2)).cuda()
    wsb = _ws_bytes(lib, "nadmm_workspace_size", _dims(lib, d), None)
    p = _params(lib, 1, 4)
    specs = {"img": (4 * V, m), "ref": (4 * V, f), "u": (12 * V, u), "v": (12 * V, v), "warped": (4 * V, None),
             "grad": (12 * V, None), "resid": (4 * V, None), "comp": (12 * V, None), "exp": (12 * V, None),
             "w": (12 * V, None), "b": (12 * V, None), "vv": (12 * V, None), "fs": (12 * V, None),
             "det": (4 * V, None), "stats": (24, None), "nneg": (8, None), "det2": (4 * V, None),
             "stats2": (24, None), "nneg2": (8, None), "ws": (wsb, None)}

    def call(b):
        s, D = _stream(), _dims(lib, d)
        wsz = ctypes.c_size_t(wsb)
        lib.call("nadmm_warp", D, b["img"].ptr(), b["u"].ptr(), b["ref"].ptr(), b["warped"].ptr(),
                 b["grad"].ptr(), b["resid"].ptr(), s)
        lib.call("nadmm_compose", D, b["u"].ptr(), b["v"].ptr(), b["comp"].ptr(), s)
        lib.call("nadmm_expmap", D, b["v"].ptr(), ctypes.c_int32(4), b["exp"].ptr(), b["ws"].ptr(), wsz, s)
        lib.call("nadmm_admm", D, ctypes.byref(p), b["grad"].ptr(), b["resid"].ptr(), b["w"].ptr(), b["b"].ptr(),
                 b["vv"].ptr(), b["ws"].ptr(), wsz, s)
        lib.call("nadmm_fourier_solve", D, ctypes.byref(p), b["v"].ptr(), b["fs"].ptr(), b["ws"].ptr(), wsz, s)
        lib.call("nadmm_jacobian", D, b["comp"].ptr(), b["det"].ptr(), b["stats"].ptr(), b["nneg"].ptr(),
                 b["ws"].ptr(), wsz, s)
        lib.call("nadmm_jacobian_noalloc", D, b["comp"].ptr(), b["det2"].ptr(), b["stats2"].ptr(),
                 b["nneg2"].ptr(), s)
    _run_both(call, specs)
