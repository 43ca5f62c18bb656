"""Writes the stored oracle expectations used by the full-size GPU parity test.

Calls only the FP64 oracle (and the seeded input generators): it runs the
whole 128x128x96 heart-phantom registration (10 warpings x 20 iterations,
n = 2, lambda = 0.01, theta = 0.1) and stores, for a fixed seeded sample of
voxels, the oracle's displacement and warped intensity, plus the Jacobian
statistics of the whole displacement and a checksum of the inputs.

    python tests/golden/make_golden.py        (about a minute on one core)
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

NAME = "phantom128x128x96"
NSAMPLE = 2048


def input_digest(pair) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pair.fixed, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(pair.moving, dtype=np.float32).tobytes())
    return h.hexdigest()


def sample_indices(shape, n, seed=7):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(shape)), size=n, replace=False))


def main():
    w = synth.WORKLOADS[NAME]
    pair = synth.make_pair(NAME)
    res = O.register(pair.fixed.astype(np.float64), pair.moving.astype(np.float64), w["lam"],
                     w["theta"], w["order"], w["outer"], w["iters"])
    idx = sample_indices(pair.fixed.shape, NSAMPLE)
    disp = res.disp.reshape(3, -1)[:, idx]
    warped = res.warped.reshape(-1)[idx]
    mn, mx, mean, nneg = O.jacobian_stats(res.disp)
    out = {
        "workload": NAME,
        "source": "oracle.register (FP64 NumPy), whole registration; values at sampled voxels",
        "params": {k: w[k] for k in ("lam", "theta", "order", "outer", "iters")},
        "input_sha256": input_digest(pair),
        "sample_seed": 7,
        "indices": idx.tolist(),
        "disp": [[float(f"{v:.10g}") for v in row] for row in disp],
        "warped": [float(f"{v:.10g}") for v in warped],
        "jacobian": {"min": mn, "max": mx, "mean": mean, "n_nonpos": nneg,
                     "n_abs_below_1e-2": int(np.count_nonzero(np.abs(O.jacobian_det(res.disp)) < 1e-2))},
        "ssd_before": O.ssd(pair.fixed, pair.moving),
        "ssd_after": O.ssd(pair.fixed, res.warped),
    }
    path = os.path.join(HERE, f"{NAME}_oracle_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, out["jacobian"], out["ssd_before"], out["ssd_after"])


if __name__ == "__main__":
    main()
