"""Calls from several host threads (the boundary's threading contract): two
threads each register their own pairs on their own stream with their own
workspace, while a third pins and autotunes launch shapes of the same size
and the timing instrumentation records every launch; every result equals
the same call made alone, bit for bit, and the timing records count the
launches of both threads."""
import threading

import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D = (64, 48, 32)
ARGS = (0.01, 0.1, 2, 3, 6)  # lambda, theta, order, warpings, iterations


@pytest.fixture(scope="module")
def api():
    from paper_2109_12688_amd import api as A
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A._lib.load()
    return A


def _pairs(seed):
    out = []
    for i in range(3):
        f = torch.from_numpy(synth.random_volume(D, seed=seed + 2 * i, smooth_kmax=3)).cuda()
        m = torch.from_numpy(synth.random_volume(D, seed=seed + 2 * i + 1, smooth_kmax=3)).cuda()
        out.append((f, m))
    return out


def test_threads_register_concurrently(api):
    from paper_2109_12688_amd import _lib
    jobs = {0: _pairs(700), 1: _pairs(720)}
    shp = tuple(jobs[0][0][0].shape)
    alone = {}
    for t, pairs in jobs.items():
        alone[t] = []
        for f, m in pairs:
            r = api.register(f, m, *ARGS)
            alone[t].append((r["disp"].clone(), r["warped"].clone()))
    torch.cuda.synchronize()
    _lib.profile_read()  # drop older records
    _lib.profile_enable(True)
    results = {0: [], 1: []}
    errors = []
    start = threading.Barrier(3)

    def worker(t):
        try:
            stream = torch.cuda.Stream()
            ws = api.workspace(shp)
            start.wait()
            with torch.cuda.stream(stream):
                for _ in range(3):
                    for f, m in jobs[t]:
                        r = api.register(f, m, *ARGS, ws=ws)
                        results[t].append((r["disp"].clone(), r["warped"].clone()))
            stream.synchronize()
        except Exception as e:  # reported below, in the main thread
            errors.append(repr(e))

    def tuner():
        try:
            ws = api.workspace(shp)
            start.wait()
            for shapes in ((2, 4, 0), (8, 2, 0), (0, 0, 0)):
                api.set_shapes(shp, *shapes)
            api.autotune(shp, ARGS[0], ARGS[1], ARGS[2], ws=ws)
        except Exception as e:
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(t,)) for t in (0, 1)] + [threading.Thread(target=tuner)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads), "a thread did not finish"
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    api.set_shapes(shp)
    assert not errors, errors
    for t in (0, 1):
        assert len(results[t]) == 9
        for i, (d, w) in enumerate(results[t]):
            ref_d, ref_w = alone[t][i % 3]
            assert torch.equal(d, ref_d) and torch.equal(w, ref_w), (t, i)
    # both threads' registrations are in the records: per registration one
    # first pass and one composition per warping
    assert prof["pass_c_compose"][0] >= 2 * 9 * ARGS[3]
    assert prof["pass_a_fwd_x"][0] >= 2 * 9 * ARGS[3]
