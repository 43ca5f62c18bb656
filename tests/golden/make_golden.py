"""Writes the stored oracle expectations used by the full-size GPU parity tests.

Calls only the FP64 oracle (and the seeded input generators).

* phantom128x128x96: the whole 128x128x96 heart-phantom registration
  (10 warpings x 20 iterations, n = 2, lambda = 0.01, theta = 0.1) on the
  float32 images.
* phantom192x192x128: the 192x192x128 phantom (10 x 30, n = 3,
  lambda = 0.005, theta = 0.1) whose images are stored as bfloat16: the
  registration of the bfloat16-rounded images (what the GPU's bfloat16 path
  must match), and of the float32 images (to report what the storage
  precision costs).

For each run: the displacement and warped intensity at a fixed seeded sample
of voxels, the Jacobian statistics of the whole displacement, SSD before and
after, and a checksum of the inputs.

* blobs96: the 96^3 blob pair's one-warping image match (20 iterations,
  n = 2, lambda = 0.01, theta = 0.1): loss, dL/dlambda and dL/dI1 at the
  sampled voxels and at 16 further seeded voxels (the finite-difference
  probes of the GPU test).

    python tests/golden/make_golden.py [phantom128x128x96 | phantom192x192x128 | blobs96]
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402

NSAMPLE = 2048


def input_digest(fixed, moving) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(fixed).tobytes())
    h.update(np.ascontiguousarray(moving).tobytes())
    return h.hexdigest()


def sample_indices(shape, n, seed=7):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(shape)), size=n, replace=False))


def run(w, fixed, moving, idx):
    res = O.register(fixed.astype(np.float64), moving.astype(np.float64), w["lam"], w["theta"],
                     w["order"], w["outer"], w["iters"])
    mn, mx, mean, nneg = O.jacobian_stats(res.disp)
    return {
        "disp": [[float(f"{v:.10g}") for v in row] for row in res.disp.reshape(3, -1)[:, idx]],
        "warped": [float(f"{v:.10g}") for v in res.warped.reshape(-1)[idx]],
        "jacobian": {"min": mn, "max": mx, "mean": mean, "n_nonpos": nneg,
                     "n_abs_below_1e-2": int(np.count_nonzero(np.abs(O.jacobian_det(res.disp)) < 1e-2))},
        "ssd_before": O.ssd(fixed, moving),
        "ssd_after": O.ssd(fixed, res.warped),
    }


def main(name):
    w = synth.WORKLOADS[name]
    pair = synth.make_pair(name)
    idx = sample_indices(pair.fixed.shape, NSAMPLE)
    out = {"workload": name, "params": {k: w[k] for k in ("lam", "theta", "order", "outer", "iters")},
           "sample_seed": 7, "indices": idx.tolist()}
    if name == "blobs96":
        rng = np.random.default_rng(31)
        fd_idx = np.sort(rng.choice(int(np.prod(pair.fixed.shape)), size=16, replace=False))
        loss, gm, gl = O.ssd_one_warping_grad(pair.fixed, pair.moving, w["lam"], w["theta"],
                                              w["order"], w["iters"])
        out["source"] = ("oracle.ssd_one_warping_grad (FP64 NumPy, reverse mode through the "
                         "iterations): loss, dL/dlambda and dL/dmoving at sampled voxels")
        out["input_sha256"] = input_digest(pair.fixed.astype(np.float32), pair.moving.astype(np.float32))
        out["loss"] = loss
        out["d_lambda"] = gl
        out["d_moving"] = [float(f"{v:.12g}") for v in gm.reshape(-1)[idx]]
        out["fd_indices"] = fd_idx.tolist()
        out["d_moving_fd_indices"] = [float(f"{v:.12g}") for v in gm.reshape(-1)[fd_idx]]
        # central differences of the FP64 loss, eps = 1e-3, at the same voxels and lambda
        eps = 1e-3
        args = (w["theta"], w["order"], w["iters"])
        mf = pair.moving.astype(np.float64).reshape(-1)
        fd = []
        for i in fd_idx:
            mp, mm = mf.copy(), mf.copy()
            mp[i] += eps
            mm[i] -= eps
            lp = O.ssd_one_warping(pair.fixed, mp.reshape(pair.moving.shape), w["lam"], *args)
            lm = O.ssd_one_warping(pair.fixed, mm.reshape(pair.moving.shape), w["lam"], *args)
            fd.append((lp - lm) / (2 * eps))
        out["fd_moving_eps1e-3"] = fd
        out["fd_lambda_eps1e-3"] = (O.ssd_one_warping(pair.fixed, pair.moving, w["lam"] + eps, *args)
                                    - O.ssd_one_warping(pair.fixed, pair.moving, w["lam"] - eps, *args)) / (2 * eps)
    elif name == "phantom192x192x128":
        fb, mb = synth.bf16_bits(pair.fixed), synth.bf16_bits(pair.moving)
        out["source"] = ("oracle.register (FP64 NumPy), whole registration; 'bf16': on the "
                         "bfloat16-rounded images, 'fp32': on the float32 images")
        out["input_sha256"] = input_digest(fb, mb)
        out["bf16"] = run(w, synth.bf16_to_f32(fb), synth.bf16_to_f32(mb), idx)
        out["fp32"] = run(w, pair.fixed, pair.moving, idx)
    else:
        out["source"] = "oracle.register (FP64 NumPy), whole registration; values at sampled voxels"
        out["input_sha256"] = input_digest(pair.fixed.astype(np.float32), pair.moving.astype(np.float32))
        r = run(w, pair.fixed, pair.moving, idx)
        out.update(r)
    path = os.path.join(HERE, f"{name}_oracle_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "phantom128x128x96")
