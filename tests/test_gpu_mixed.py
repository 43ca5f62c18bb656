"""Pairs of several sizes in one call (nadmm_register_mixed: one launch per
phase over every pair of every size), through the C ABI: each pair bit for
bit equal to its own nadmm_register call, pairs of the batching workload's
three sizes among them, and a batch whose y-z workgroups each transform two
or more small planes; one pair of each of two sizes against the FP64
oracle; the call captured in a graph and replayed; argument errors."""
import ctypes

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAM, THETA, ORDER = 0.01, 0.1, 2


@pytest.fixture(scope="module")
def api():
    from paper_2109_12688_amd import api as A
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A._lib.load()
    return A


def _pair(dims_xyz, seed):
    f = synth.random_volume(dims_xyz, seed=seed, smooth_kmax=3)
    m = synth.random_volume(dims_xyz, seed=seed + 1, smooth_kmax=3)
    return torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()


def _singles(api, pairs, outer, iters):
    out = []
    for f, m in pairs:
        r = api.register(f, m, LAM, THETA, ORDER, outer, iters)
        out.append((r["disp"].clone(), r["warped"].clone()))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("case", ["small", "batching_sizes"])
def test_mixed_equals_single_calls(api, case):
    if case == "small":
        # four sizes, one of them twice, pairs not grouped by size
        sizes = [(64, 32, 32), (96, 32, 64), (64, 32, 32), (128, 64, 32), (64, 64, 32)]
        outer, iters = 2, 4
    else:
        sizes = [(128, 128, 96), (64, 64, 64), (96, 96, 64), (64, 64, 64)]
        outer, iters = 2, 3
    pairs = [_pair(d, 500 + 2 * i) for i, d in enumerate(sizes)]
    ref = _singles(api, pairs, outer, iters)
    res = api.register_mixed([p[0] for p in pairs], [p[1] for p in pairs], LAM, THETA, ORDER, outer, iters)
    torch.cuda.synchronize()
    for i, (d, w) in enumerate(ref):
        assert torch.equal(res["disp"][i], d), f"pair {i} {sizes[i]}: displacement differs"
        assert torch.equal(res["warped"][i], w), f"pair {i} {sizes[i]}: warped image differs"


def test_mixed_against_oracle(api):
    sizes = [(64, 32, 32), (96, 32, 64)]
    outer, iters = 2, 5
    pairs = [_pair(d, 520 + 2 * i) for i, d in enumerate(sizes)]
    res = api.register_mixed([p[0] for p in pairs], [p[1] for p in pairs], LAM, THETA, ORDER, outer, iters)
    torch.cuda.synchronize()
    for i, (f, m) in enumerate(pairs):
        ref = O.register(f.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64), LAM, THETA,
                         ORDER, outer, iters)
        derr = np.abs(res["disp"][i].cpu().numpy() - ref.disp).max()
        werr = np.abs(res["warped"][i].cpu().numpy() - ref.warped).max()
        assert derr < 1e-3 and werr < 1e-4, (sizes[i], derr, werr)


def test_mixed_graph_replay(api):
    sizes = [(64, 32, 32), (96, 32, 64), (64, 64, 32)]
    outer, iters = 2, 3
    pairs = [_pair(d, 540 + 2 * i) for i, d in enumerate(sizes)]
    fl, ml = [p[0] for p in pairs], [p[1] for p in pairs]
    ws = api.workspace_mixed([tuple(f.shape) for f in fl])
    eager = api.register_mixed(fl, ml, LAM, THETA, ORDER, outer, iters, ws=ws)
    torch.cuda.synchronize()
    ref_d = eager["packed"][2].clone()
    ref_w = eager["packed"][3].clone()
    packed = tuple(t for t in eager["packed"])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        api.register_mixed(fl, ml, LAM, THETA, ORDER, outer, iters, ws=ws, packed=packed)
    torch.cuda.synchronize()
    for _ in range(3):
        packed[2].fill_(0.0)
        packed[3].fill_(-1.0)
        ws.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(packed[2], ref_d) and torch.equal(packed[3], ref_w)


def test_mixed_no_warping(api):
    sizes = [(64, 32, 32), (96, 32, 64)]
    pairs = [_pair(d, 560 + 2 * i) for i, d in enumerate(sizes)]
    res = api.register_mixed([p[0] for p in pairs], [p[1] for p in pairs], LAM, THETA, ORDER, 0, 3)
    torch.cuda.synchronize()
    for i, (f, m) in enumerate(pairs):
        assert torch.count_nonzero(res["disp"][i]) == 0
        assert torch.equal(res["warped"][i], m)


def test_mixed_rejects_bad_arguments(api):
    L = api._lib.load()
    n = ctypes.c_size_t(0)
    d = (api.Dims * 2)(api.Dims(32, 32, 32), api.Dims(64, 32, 32))
    assert L.nadmm_workspace_size_mixed(2, d, ctypes.byref(n)) == 2  # nx = 32 has no mixed code
    assert "nx in" in L.nadmm_last_error().decode()
    nine = [(64, 32, 32), (64, 32, 64), (64, 32, 96), (64, 32, 128), (64, 64, 32), (64, 64, 64), (64, 64, 96),
            (64, 64, 128), (64, 96, 32)]
    many = (api.Dims * 9)(*[api.Dims(*t) for t in nine])
    assert L.nadmm_workspace_size_mixed(8, many, ctypes.byref(n)) == 0
    assert L.nadmm_workspace_size_mixed(9, many, ctypes.byref(n)) == 1  # more than 8 sizes
    assert L.nadmm_workspace_size_mixed(0, d, ctypes.byref(n)) == 1
    assert L.nadmm_workspace_size_mixed(1, d, ctypes.byref(n)) == 2
    split = (api.Dims * 3)(api.Dims(64, 32, 32), api.Dims(96, 32, 64), api.Dims(64, 32, 32))
    assert L.nadmm_workspace_size_mixed(3, split, ctypes.byref(n)) == 1  # a size's pairs not consecutive
    assert "consecutive" in L.nadmm_last_error().decode()
