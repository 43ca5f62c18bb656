"""nadmm_jacobian_noalloc (no workspace; the reduction's partials in the
library's own device array) against nadmm_jacobian, through the C ABI: the
same determinant map, statistics and count, bit for bit, on two calls in a
row, the second with a smaller field, and again with the map not requested."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2109_12688_amd import _lib
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _lib


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _run(lib, fn, disp, want_det, ws=None):
    nz, ny, nx = disp.shape[1:]
    d = lib.Dims(nx, ny, nz)
    det = torch.full((nz, ny, nx), float("nan"), dtype=torch.float32, device="cuda") if want_det else None
    stats = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    nneg = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if fn == "nadmm_jacobian":
        lib.call(fn, d, _ptr(disp), _ptr(det), _ptr(stats), _ptr(nneg), _ptr(ws),
                 ctypes.c_size_t(ws.numel()), stream)
    else:
        lib.call(fn, d, _ptr(disp), _ptr(det), _ptr(stats), _ptr(nneg), stream)
    torch.cuda.synchronize()
    return (None if det is None else det.cpu().numpy()), stats.cpu().numpy(), int(nneg.cpu()[0])


def _workspace(lib, disp):
    nz, ny, nx = disp.shape[1:]
    n = ctypes.c_size_t(0)
    lib.check("nadmm_workspace_size", lib.load().nadmm_workspace_size(lib.Dims(nx, ny, nz), None,
                                                                        ctypes.byref(n)))
    return torch.empty(n.value, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("want_det", [True, False])
def test_noalloc_equals_workspace_entry_point(lib, want_det):
    lib.load()
    # uniform noise displacements (they fold: many det <= 0) on a grid that
    # fills all 1024 reduction blocks, then a smaller grid of 21 blocks
    cases = [((96, 64, 48), 3.0, 11), ((24, 18, 12), 1.5, 12)]
    for dims, amp, seed in cases:
        u = synth.random_vector_field(dims, seed=seed, amp=amp)
        disp = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float32)).cuda()
        ws = _workspace(lib, disp)
        ref = _run(lib, "nadmm_jacobian", disp, want_det, ws)
        got = _run(lib, "nadmm_jacobian_noalloc", disp, want_det)
        if want_det:
            assert np.array_equal(got[0].view(np.uint32), ref[0].view(np.uint32)), dims
        assert np.array_equal(got[1].view(np.uint64), ref[1].view(np.uint64)), (dims, got[1], ref[1])
        assert got[2] == ref[2], dims
        assert np.isfinite(got[1]).all() and got[2] >= 0
    # the first case folds, so the count compared above is not trivially 0
    u = synth.random_vector_field(cases[0][0], seed=cases[0][2], amp=cases[0][1])
    disp = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float32)).cuda()
    assert _run(lib, "nadmm_jacobian_noalloc", disp, False)[2] > 0


def test_noalloc_rejects_bad_arguments_without_launching(lib):
    L = lib.load()
    dummy = torch.zeros(4, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.nadmm_jacobian_noalloc(lib.Dims(10, 8, 8), p, None, p, p, stream) == 2  # unsupported size
    assert L.nadmm_jacobian_noalloc(lib.Dims(8, 8, 8), None, None, p, p, stream) == 1  # NULL disp
    assert "NULL" in L.nadmm_last_error().decode()
