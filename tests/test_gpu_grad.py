"""GPU parity of the differentiated warping (nadmm_ssd_grad).

L = sum (I1(x + w(x)) - I0(x))^2, w the velocity of one warping of `iters`
unrolled Nesterov-ADMM iterations.  The GPU gradient (reverse pass in the
library's kernels, float32 fields, float64 reductions) is compared with the
FP64 oracle's adjoint (reverse mode through the literal recurrence of
Eq. (5)) at every voxel on small grids, with itself across checkpoint
intervals, with torch.autograd through the Function wrapper, and at the 96^3
blob workload with central differences (eps = 1e-3 on 16 voxels and on
lambda) and the stored oracle gradient.

Tolerances: the loss to 1e-4 relative (it sums squares of small residuals:
|dL| <= 2 sqrt(L V) d for a per-voxel intensity error d, which is 7e-4 of L
at 96^3 for d = 1e-6); gradients to 1e-4 of their max norm (a float32
forward and reverse pass of ~4 Fourier solves per iteration each carry ~1e-6
relative error; the bound leaves two orders of magnitude); the central
difference checks as stated in the 96^3 test.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def api():
    from paper_2109_12688_amd import api as A
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A._lib.load()
    return A


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def pair(d, seed):
    f = synth.random_volume(d, seed=seed, smooth_kmax=3)
    m = synth.random_volume(d, seed=seed + 1, smooth_kmax=3)
    return f, m


@pytest.mark.parametrize("d,order,iters,ck", [((16, 12, 9), 2, 6, 2), ((24, 18, 16), 1, 7, 3),
                                               ((12, 144, 128), 2, 4, 2), ((16, 32, 24), 2, 5, 2)])
def test_gradient_vs_oracle_adjoint(api, d, order, iters, ck):
    f, m = pair(d, 300)
    lam, theta = 0.02, 0.1
    loss, dm, dl = api.ssd_grad(gpu(f), gpu(m), lam, theta, order, iters, checkpoint=ck)
    e_loss, e_dm, e_dl = O.ssd_one_warping_grad(f.astype(np.float64), m.astype(np.float64), lam, theta,
                                                order, iters)
    assert abs(loss.item() - e_loss) < 1e-4 * e_loss
    assert np.abs(host(dm) - e_dm).max() < 1e-4 * np.abs(e_dm).max()
    assert abs(dl.item() - e_dl) < 1e-4 * max(abs(e_dl), 1e-12)


def test_checkpoint_interval_does_not_change_the_gradient(api):
    d = (16, 12, 9)
    f, m = pair(d, 310)
    outs = [api.ssd_grad(gpu(f), gpu(m), 0.01, 0.1, 2, 9, checkpoint=c) for c in (1, 2, 4, 9)]
    l0, dm0, dl0 = outs[0]
    for loss, dm, dl in outs[1:]:
        assert loss.item() == l0.item()
        assert np.abs(host(dm) - host(dm0)).max() < 1e-6 * np.abs(host(dm0)).max()
        assert abs(dl.item() - dl0.item()) < 1e-9 * abs(dl0.item())


def test_autograd_function(api):
    from paper_2109_12688_amd.autograd import one_warping_ssd
    d = (16, 12, 9)
    f, m = pair(d, 320)
    mov = gpu(m).requires_grad_(True)
    lam = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    loss = one_warping_ssd(mov, lam, gpu(f), 0.1, 2, 6, 3)
    gm, gl = torch.autograd.grad(3.0 * loss, (mov, lam))
    l2, dm, dl = api.ssd_grad(gpu(f), gpu(m), 0.01, 0.1, 2, 6, checkpoint=3)
    assert loss.item() == l2.item()
    assert np.abs(host(gm) - 3.0 * host(dm)).max() <= 1e-6 * np.abs(host(dm)).max()
    assert abs(gl.item() - 3.0 * dl.item()) <= 1e-12 * abs(dl.item())
    # no gradient required: the loss alone (no reverse pass), the same value
    with torch.no_grad():
        l3 = one_warping_ssd(gpu(m), 0.01, gpu(f), 0.1, 2, 6, 3)
    l4, n1, n2 = api.ssd_grad(gpu(f), gpu(m), 0.01, 0.1, 2, 6, checkpoint=3, loss_only=True)
    assert n1 is None and n2 is None
    assert l3.item() == l2.item() and l4.item() == l2.item()


def test_blobs96_finite_differences_and_oracle(api):
    """The 96^3 blob pair, one warping of 20 iterations, checkpoints
    every 5; eps = 1e-3 on 16 probe voxels and on lambda.  The probes are
    where the oracle's |dL/dI1| is largest (one per 8^3 block), so every
    central difference is far from zero (|dL/dI1| >= 0.07 there, against
    ~1e-10 in the flat background).

    (1) The GPU gradient against the FP64 oracle's adjoint (2048 + 16
    voxels, lambda) to 1e-4 of the max norm.  (2) Against the FP64 oracle's
    central differences: voxels to 1e-3 relative + 1e-8; lambda to 1e-2
    (eps = 1e-3 is 10 % of
    lambda = 0.01: the central difference itself is 0.37 % off the
    derivative, in FP64 as well).  (3) The GPU's own central differences of
    its float32 loss: 2e-2 relative + 5e-4 absolute (the loss moves by up to
    ~1e-6 under any one-voxel perturbation through rounding alone, i.e.
    ~5e-4 after division by 2 eps)."""
    name = "blobs96"
    w = synth.WORKLOADS[name]
    with open(os.path.join(HERE, "golden", f"{name}_oracle_samples.json")) as fh:
        gold = json.load(fh)
    p = synth.make_pair(name)
    f, m = gpu(p.fixed), gpu(p.moving)
    args = (w["lam"], w["theta"], w["order"], w["iters"])
    ws = api.workspace_grad(p.fixed.shape, *args, w["checkpoint"])
    loss, dm, dl = api.ssd_grad(f, m, *args, checkpoint=w["checkpoint"], ws=ws)
    g = host(dm).reshape(-1)
    idx = np.array(gold["indices"])
    e = np.array(gold["d_moving"])
    scale = np.abs(e).max()
    fd_idx = np.array(gold["fd_indices"])
    # (1) the oracle's adjoint
    assert abs(loss.item() - gold["loss"]) < 1e-4 * gold["loss"]
    assert abs(dl.item() - gold["d_lambda"]) < 1e-4 * abs(gold["d_lambda"])
    assert np.abs(g[idx] - e).max() < 1e-4 * scale
    assert np.abs(g[fd_idx] - np.array(gold["d_moving_fd_indices"])).max() < 1e-4 * scale
    # (2) the oracle's central differences
    fd64 = np.array(gold["fd_moving_eps1e-3"])
    assert np.abs(fd64).min() >= 1e-6  # every probe tests a derivative that is not ~0
    assert np.all(np.abs(g[fd_idx] - fd64) <= 1e-3 * np.abs(fd64) + 1e-8)
    assert abs(dl.item() - gold["fd_lambda_eps1e-3"]) < 1e-2 * abs(gold["fd_lambda_eps1e-3"])
    # (3) central differences of the GPU's own loss, eps = 1e-3
    eps = 1e-3

    def L(mov, lam):
        return api.ssd_grad(f, mov, lam, *args[1:], checkpoint=w["checkpoint"], ws=ws)[0].item()

    flat = m.reshape(-1)
    fd32 = []
    for i in fd_idx:
        old = flat[i].item()
        flat[i] = old + eps
        lp = L(m, w["lam"])
        flat[i] = old - eps
        lm = L(m, w["lam"])
        flat[i] = old
        fd32.append((lp - lm) / (2 * eps))
    fd32 = np.array(fd32)
    fd_l = (L(m, w["lam"] + eps) - L(m, w["lam"] - eps)) / (2 * eps)
    print(f"blobs96: loss {loss.item():.6f}; dL/dlambda {dl.item():.5f} (oracle adjoint "
          f"{gold['d_lambda']:.5f}, oracle central difference {gold['fd_lambda_eps1e-3']:.5f}, GPU "
          f"central difference {fd_l:.5f}); largest |dL/dI1| probe {g[fd_idx][np.argmax(np.abs(fd64))]:+.6e} "
          f"vs oracle central difference {fd64[np.argmax(np.abs(fd64))]:+.6e}; GPU central differences "
          f"within {np.abs(fd32 - g[fd_idx]).max():.2e} of the GPU gradient")
    assert np.all(np.abs(fd32 - g[fd_idx]) <= 2e-2 * np.abs(g[fd_idx]) + 5e-4)
    assert abs(fd_l - gold["fd_lambda_eps1e-3"]) < 2e-3 * abs(gold["fd_lambda_eps1e-3"])
