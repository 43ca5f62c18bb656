"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2109_12688_amd import _lib
from paper_2109_12688_amd._lib import Dims, Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nadmm.h")

FAKE = ctypes.c_void_p(0x10000)       # aligned stand-in pointer: never dereferenced on error paths
MISALIGNED = ctypes.c_void_p(0x10004)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2109_12688_amd.build import build
        build()
    return _lib.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nadmm_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_are_exported(lib):
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_library_built_from_these_sources(lib):
    """The digest compiled into the loaded library is the digest of the
    sources on disk (load() refuses a stale build)."""
    from paper_2109_12688_amd.build import source_files, sources_digest
    assert lib.nadmm_source_digest().decode() == sources_digest()
    names = [os.path.basename(f) for f in source_files()]
    assert "capi.hip" in names and "kernels.hip" in names and names[-1] == "nadmm.h"


def test_abi_version_and_status_strings(lib):
    assert lib.nadmm_abi_version() == 1
    for code, name in _lib.STATUS_NAMES.items():
        assert lib.nadmm_status_string(code).decode() == name


def _p(**kw):
    base = dict(lambda_=0.01, theta=0.1, order=2, data_term=2, eps=1e-8, outer=2, iters=3)
    base.update(kw)
    return Params(**base)


def ws_size(lib, d):
    n = ctypes.c_size_t(0)
    st = lib.nadmm_workspace_size(d, None, ctypes.byref(n))
    return st, n.value


def test_workspace_size(lib):
    st, n = ws_size(lib, Dims(128, 128, 96))
    assert st == 0
    V = 128 * 128 * 96
    # 14 float32 fields of V voxels, the extra Nyquist plane of the half
    # spectrum (3 components x ny*nz complex), plus transform tables
    base = 14 * 4 * V + 3 * 128 * 96 * 8
    assert base <= n <= base + 64 * 1024
    assert lib.nadmm_workspace_size(Dims(128, 128, 96), None, None) == 1


@pytest.mark.parametrize("d", [(32, 256, 96), (192, 192, 128), (256, 256, 256), (12, 162, 128)])
def test_large_planes_supported(lib, d):
    st, n = ws_size(lib, Dims(*d))
    assert st == 0, lib.nadmm_last_error()
    assert n >= 14 * 4 * d[0] * d[1] * d[2]


@pytest.mark.parametrize("d", [(128, 128, 7), (6, 4, 4), (128, 129, 96), (512, 16, 16),
                               (32, 250, 96), (0, 8, 8), (-8, 8, 8), (4, 4, 2)])
def test_unsupported_sizes(lib, d):
    st, _ = ws_size(lib, Dims(*d))
    assert st == 2, lib.nadmm_last_error()
    p = _p()
    st = lib.nadmm_register(Dims(*d), ctypes.byref(p), FAKE, FAKE, None, FAKE, None, None, FAKE,
                            1 << 40, None)
    assert st == 2
    assert b"dims" in lib.nadmm_last_error()


@pytest.mark.parametrize("kw", [dict(theta=0.0), dict(theta=-1.0), dict(theta=float("nan")),
                                dict(lambda_=-0.1), dict(lambda_=float("inf")), dict(order=0),
                                dict(order=5), dict(data_term=3), dict(data_term=1, eps=0.0),
                                dict(iters=0), dict(outer=-1)])
def test_bad_params(lib, kw):
    p = _p(**kw)
    d = Dims(32, 32, 32)
    st = lib.nadmm_register(d, ctypes.byref(p), FAKE, FAKE, None, FAKE, None, None, FAKE, 1 << 40, None)
    assert st == 1, lib.nadmm_last_error()


def test_null_and_misaligned_pointers(lib):
    p = _p()
    d = Dims(32, 32, 32)
    big = ctypes.c_size_t(1 << 40)
    assert lib.nadmm_register(d, None, FAKE, FAKE, None, FAKE, None, None, FAKE, big, None) == 1
    assert lib.nadmm_register(d, ctypes.byref(p), None, FAKE, None, FAKE, None, None, FAKE, big, None) == 1
    assert lib.nadmm_register(d, ctypes.byref(p), FAKE, MISALIGNED, None, FAKE, None, None, FAKE, big, None) == 1
    assert b"aligned" in lib.nadmm_last_error()
    assert lib.nadmm_admm(d, ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, big, None) == 1
    assert lib.nadmm_warp(d, FAKE, FAKE, None, FAKE, None, FAKE, None) == 1  # resid needs ref
    assert lib.nadmm_compose(d, FAKE, ctypes.c_void_p(0x20000), FAKE, None) == 1  # out aliases u
    assert lib.nadmm_expmap(d, FAKE, 31, ctypes.c_void_p(0x20000), FAKE, big, None) == 1
    assert lib.nadmm_expmap(d, FAKE, 3, FAKE, FAKE, big, None) == 1  # out aliases vel


def test_count_nonfinite_argument_checks(lib):
    d = Dims(32, 32, 32)
    assert lib.nadmm_count_nonfinite(d, None, 3, FAKE, None) == 1
    assert lib.nadmm_count_nonfinite(d, FAKE, 3, None, None) == 1
    assert lib.nadmm_count_nonfinite(d, MISALIGNED, 1, FAKE, None) == 1
    assert lib.nadmm_count_nonfinite(d, FAKE, 0, FAKE, None) == 1
    assert lib.nadmm_count_nonfinite(d, FAKE, 65, FAKE, None) == 1
    assert lib.nadmm_count_nonfinite(Dims(30, 32, 32), FAKE, 1, FAKE, None) == 2


def test_register_threshold_argument_checks(lib):
    p = _p()
    d = Dims(32, 32, 32)
    _, need = ws_size(lib, d)
    n = ctypes.c_size_t(need)
    nan, tol = ctypes.c_double(float("nan")), ctypes.c_double(0.05)

    def call(d=d, ta=tol, tw=tol, fixed=FAKE, disp=FAKE, ws_bytes=n):
        return lib.nadmm_register_threshold(d, ctypes.byref(p), ta, tw, fixed, FAKE, disp, None, None, None,
                                            None, None, FAKE, ws_bytes, None)
    assert call(ta=nan) == 1
    assert call(tw=nan) == 1
    assert call(fixed=None) == 1
    assert call(disp=MISALIGNED) == 1
    assert call(ws_bytes=ctypes.c_size_t(need - 1)) == 3
    assert call(d=Dims(30, 32, 32)) == 2


def test_register_pyramid_threshold_argument_checks(lib):
    p = _p()
    d = Dims(32, 32, 32)
    py = _lib.Pyramid(3, (2, 2, 1, 0), (3, 2, 2, 0))
    need = ctypes.c_size_t(0)
    assert lib.nadmm_workspace_size_pyramid(d, ctypes.byref(py), ctypes.byref(need)) == 0
    n = ctypes.c_size_t(need.value)
    nan, tol = ctypes.c_double(float("nan")), ctypes.c_double(0.05)

    def call(d=d, pyr=py, ta=tol, fixed=FAKE, ws_bytes=n):
        return lib.nadmm_register_pyramid_threshold(d, ctypes.byref(p), ctypes.byref(pyr) if pyr else None, ta,
                                                    tol, fixed, FAKE, FAKE, None, None, None, FAKE, ws_bytes,
                                                    None)
    assert call(ta=nan) == 1
    assert call(fixed=None) == 1
    assert call(pyr=None) == 1
    assert call(ws_bytes=ctypes.c_size_t(need.value - 1)) == 3
    bad = _lib.Pyramid(5, (1, 1, 1, 1), (1, 1, 1, 1))
    assert call(pyr=bad) == 1


def test_workspace_too_small(lib):
    p = _p()
    d = Dims(32, 32, 32)
    _, need = ws_size(lib, d)
    st = lib.nadmm_register(d, ctypes.byref(p), FAKE, FAKE, None, FAKE, None, None, FAKE,
                            ctypes.c_size_t(need - 1), None)
    assert st == 3
    assert lib.nadmm_admm(d, ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, need, None) == 1
    st = lib.nadmm_jacobian(d, FAKE, None, FAKE, FAKE, FAKE, ctypes.c_size_t(16), None)
    assert st == 3
    st = lib.nadmm_fourier_solve(d, ctypes.byref(p), FAKE, FAKE, FAKE, ctypes.c_size_t(need // 2), None)
    assert st == 3


def test_profile_read_without_records(lib):
    assert lib.nadmm_profile_enable(0) == 0
    prof = _lib.profile_read()
    assert prof == {}


def test_python_binding_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_2109_12688_amd import api
    x = torch.zeros(4, 4, 8)
    with pytest.raises(ValueError):
        api.warp(x, torch.zeros(3, 4, 4, 8))


def test_pyramid_argument_checks(lib):
    from paper_2109_12688_amd._lib import Pyramid
    n = ctypes.c_size_t(0)
    py = Pyramid()
    py.levels = 3
    for i, (o, k) in enumerate(((10, 10), (10, 5), (5, 5))):
        py.outer[i], py.iters[i] = o, k
    assert lib.nadmm_workspace_size_pyramid(Dims(128, 128, 96), ctypes.byref(py), ctypes.byref(n)) == 0
    assert n.value > 14 * 4 * 128 * 128 * 96
    # 100 is not divisible by 4 for three levels; 4 levels of 24^3 reach 3^3
    assert lib.nadmm_workspace_size_pyramid(Dims(100, 128, 96), ctypes.byref(py), ctypes.byref(n)) == 2
    py.levels = 4
    py.outer[3], py.iters[3] = 1, 1
    assert lib.nadmm_workspace_size_pyramid(Dims(24, 24, 24), ctypes.byref(py), ctypes.byref(n)) == 2
    py.levels = 5
    assert lib.nadmm_workspace_size_pyramid(Dims(64, 64, 64), ctypes.byref(py), ctypes.byref(n)) == 1


def test_set_shapes_pins_and_validates(lib):
    """nadmm_set_shapes (host tables only): valid shapes read back through
    nadmm_tuned_shapes, invalid ones are rejected and change nothing, and 0
    restores the defaults."""
    d = Dims(128, 128, 96)
    out = (ctypes.c_int32 * 3)()
    assert lib.nadmm_tuned_shapes(d, out) == 0
    default = list(out)
    assert lib.nadmm_set_shapes(d, (ctypes.c_int32 * 3)(16, 4, 1024)) == 0
    assert lib.nadmm_tuned_shapes(d, out) == 0 and list(out) == [16, 4, 1024]
    for bad in ([6, 4, 1024], [34, 4, 1024], [16, 3, 1024], [16, 4, 1000], [16, 4, 2048], [16, 4, 64],
                [-2, 4, 1024]):
        assert lib.nadmm_set_shapes(d, (ctypes.c_int32 * 3)(*bad)) == 1, bad
        assert lib.nadmm_tuned_shapes(d, out) == 0 and list(out) == [16, 4, 1024], bad
    assert "shape" in lib.nadmm_last_error().decode() or "rows" in lib.nadmm_last_error().decode()
    assert lib.nadmm_set_shapes(d, None) == 1
    # planes of 192 x 128 take the three-launch path: no plane threads to set
    big = Dims(192, 192, 128)
    assert lib.nadmm_set_shapes(big, (ctypes.c_int32 * 3)(0, 0, 256)) == 1
    assert lib.nadmm_set_shapes(big, (ctypes.c_int32 * 3)(8, 8, 0)) == 0
    # 24 or 32 rows of 192-point lines would need more threads than the x-line
    # kernels' launch bound of 768: rejected, x-line and composition rows alike
    for rows in (24, 32):
        assert lib.nadmm_set_shapes(big, (ctypes.c_int32 * 3)(rows, 8, 0)) == 1, rows
        assert lib.nadmm_set_shapes(big, (ctypes.c_int32 * 3)(8, rows, 0)) == 1, rows
    assert lib.nadmm_set_shapes(big, (ctypes.c_int32 * 3)(16, 12, 0)) == 0
    assert lib.nadmm_set_shapes(big, (ctypes.c_int32 * 3)(0, 0, 0)) == 0
    assert lib.nadmm_set_shapes(d, (ctypes.c_int32 * 3)(0, 0, 0)) == 0
    assert lib.nadmm_tuned_shapes(d, out) == 0 and list(out) == default
