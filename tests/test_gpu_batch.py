"""GPU parity of the batched registration (nadmm_register_batch): every pair
of a batch must come out bit for bit as from its own nadmm_register call
(the batch only adds a grid dimension), at a one-pass and at a half-plane
size; one pair is also checked against the FP64 oracle."""
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


@pytest.mark.parametrize("d,b", [((32, 24, 16), 3), ((8, 144, 128), 2), ((64, 64, 64), 2)])
def test_batch_equals_single_calls(api, d, b):
    f = np.stack([synth.random_volume(d, seed=60 + i, smooth_kmax=3) for i in range(b)])
    m = np.stack([synth.random_volume(d, seed=80 + i, smooth_kmax=3) for i in range(b)])
    lam, theta, order, outer, iters = 0.01, 0.1, 2, 3, 6
    res = api.register_batch(gpu(f), gpu(m), lam, theta, order, outer, iters)
    for i in range(b):
        one = api.register(gpu(f[i]), gpu(m[i]), lam, theta, order, outer, iters)
        assert torch.equal(res["disp"][i], one["disp"]), i
        assert torch.equal(res["warped"][i], one["warped"]), i


def test_batch_pair_vs_oracle(api):
    d = (32, 24, 16)
    f = np.stack([synth.random_volume(d, seed=90 + i, smooth_kmax=3) for i in range(2)])
    m = np.stack([synth.random_volume(d, seed=95 + i, smooth_kmax=3) for i in range(2)])
    res = api.register_batch(gpu(f), gpu(m), 0.02, 0.1, 2, 2, 5)
    torch.cuda.synchronize()
    ref = O.register(f[1].astype(np.float64), m[1].astype(np.float64), 0.02, 0.1, 2, 2, 5)
    assert np.abs(res["disp"][1].cpu().numpy() - ref.disp).max() < 1e-3
    assert np.abs(res["warped"][1].cpu().numpy() - ref.warped).max() < 1e-4


def test_batch_rejects_bad_batch(api):
    from paper_2109_12688_amd import _lib
    with pytest.raises(Exception):
        api.workspace_batch((16, 8, 8), 0)


def test_autotune_keeps_results(api):
    d = (32, 24, 16)
    f = gpu(synth.random_volume(d, seed=110, smooth_kmax=3))
    m = gpu(synth.random_volume(d, seed=111, smooth_kmax=3))
    args = (0.01, 0.1, 2, 2, 5)
    before = api.register(f, m, *args)
    rows = api.autotune(f.shape, 0.01, 0.1, 2)
    assert rows > 0 and d[1] % rows == 0 and rows % 2 == 0
    t = api.tuned_shapes(f.shape)
    assert t["xline_rows"] == rows
    assert d[1] % t["compose_rows"] == 0 and t["compose_rows"] % 2 == 0
    assert t["plane_threads"] % 64 == 0 and 64 <= t["plane_threads"] <= 1024
    after = api.register(f, m, *args)
    assert torch.equal(before["disp"], after["disp"])
    assert torch.equal(before["warped"], after["warped"])


def test_autotune_large_lines_stays_within_launch_bound(api):
    """Autotuning 192-point x lines (planes of 192 x 128, transformed as half
    planes) considers only rows whose workgroups fit the x-line kernels'
    768-thread launch bound (24 and 32 rows would need 864 and 1152) and
    completes; the registration is unchanged by the chosen shapes."""
    shp = (128, 192, 192)
    ws = api.workspace(shp)
    rows = api.autotune(shp, 0.005, 0.1, 3, ws=ws)
    torch.cuda.synchronize()
    t = api.tuned_shapes(shp)
    assert rows == t["xline_rows"] and rows in (2, 4, 6, 8, 12, 16)
    assert t["compose_rows"] in (2, 4, 6, 8, 12, 16) and t["plane_threads"] == 0
    api.set_shapes(shp)


def test_pinned_shapes_keep_results(api):
    """Shapes pinned with nadmm_set_shapes (non-default rows and plane
    threads) give the same registration bit for bit."""
    d = (32, 24, 16)
    f = gpu(synth.random_volume(d, seed=112, smooth_kmax=3))
    m = gpu(synth.random_volume(d, seed=113, smooth_kmax=3))
    args = (0.01, 0.1, 2, 2, 5)
    api.set_shapes(f.shape)
    before = api.register(f, m, *args)
    for shapes in ((2, 4, 0), (8, 2, 0), (4, 8, 1024)):
        api.set_shapes(f.shape, *shapes)
        t = api.tuned_shapes(f.shape)
        assert t["xline_rows"] == shapes[0] and t["compose_rows"] == shapes[1]
        after = api.register(f, m, *args)
        assert torch.equal(before["disp"], after["disp"]), shapes
        assert torch.equal(before["warped"], after["warped"]), shapes
    api.set_shapes(f.shape)


def test_graph_replay_matches_eager(api):
    """A registration captured in a graph: several replays, with eager work
    and synchronisations between them, each equal to the eager result."""
    d = (32, 24, 16)
    f = gpu(synth.random_volume(d, seed=120, smooth_kmax=3))
    m = gpu(synth.random_volume(d, seed=121, smooth_kmax=3))
    args = (0.01, 0.1, 2, 3, 6)
    shp = tuple(f.shape)
    ws = api.workspace(shp)
    out = {"disp": torch.empty((3,) + shp, device="cuda"), "warped": torch.empty(shp, device="cuda")}
    api.register(f, m, *args, ws=ws, out=out)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in out.items()}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        api.register(f, m, *args, ws=ws, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.register(f, m, *args, ws=ws, out=out)
    other = gpu(synth.random_volume(d, seed=122, smooth_kmax=3))
    for _ in range(3):
        out["disp"].zero_()
        out["warped"].zero_()
        api.register(other, m, *args)  # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["disp"], eager["disp"])
        assert torch.equal(out["warped"], eager["warped"])
