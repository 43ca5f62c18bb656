"""Writes the stored oracle expectations used by the full-size GPU parity tests.

Calls only the FP64 oracle (and the seeded input generators).

* phantom128x128x96: the whole 128x128x96 heart-phantom registration
  (10 warpings x 20 iterations, n = 2, lambda = 0.01, theta = 0.1) on the
  float32 images.
* phantom192x192x128: the 192x192x128 phantom (10 x 30, n = 3,
  lambda = 0.005, theta = 0.1) whose images are stored as bfloat16: the
  registration of the bfloat16-rounded images (what the GPU's bfloat16 path
  must match), and of the float32 images (to report what the storage
  precision costs).  16384 uniformly drawn voxels plus 2048 voxels drawn
  from the neighbourhoods of the float32-image oracle's folds (voxels whose
  9x9x9 periodic neighbourhood holds a determinant <= 0.1); for every sample
  and both runs, that neighbourhood minimum of the oracle's determinant; and
  for both runs the full-field distance of a float32 run of the same steps
  (fp32_mirror.py) from the FP64 oracle.

For each run: the displacement and warped intensity at a fixed seeded sample
of voxels, the Jacobian statistics of the whole displacement, SSD before and
after, and a checksum of the inputs.

* blobs96: the 96^3 blob pair's one-warping image match (20 iterations,
  n = 2, lambda = 0.01, theta = 0.1): loss, dL/dlambda and dL/dI1 at the
  sampled voxels and at 16 finite-difference probe voxels: those with the
  largest |dL/dI1| of the oracle, one per 8^3 block so that they spread over
  the image (the central differences of the GPU test then test something:
  in the flat background the derivative is ~1e-10).

    python tests/golden/make_golden.py [phantom128x128x96 | phantom192x192x128 | blobs96]
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
import synth  # noqa: E402

NSAMPLE = 2048
NSAMPLE_192 = 16384
NFOLD_192 = 2048
FOLD_DET = 0.1


def input_digest(fixed, moving) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(fixed).tobytes())
    h.update(np.ascontiguousarray(moving).tobytes())
    return h.hexdigest()


def sample_indices(shape, n, seed=7):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(shape)), size=n, replace=False))


def nbhd_min_det(disp):
    """Minimum of the oracle's det(I + Du) over the 9x9x9 periodic
    neighbourhood of every voxel."""
    from scipy import ndimage
    return ndimage.minimum_filter(O.jacobian_det(disp), size=9, mode="wrap")


def oracle_register(w, fixed, moving):
    return O.register(fixed.astype(np.float64), moving.astype(np.float64), w["lam"], w["theta"],
                      w["order"], w["outer"], w["iters"])


def run(w, fixed, moving, idx, res=None):
    if res is None:
        res = oracle_register(w, fixed, moving)
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
    idx = sample_indices(pair.fixed.shape, NSAMPLE_192 if name == "phantom192x192x128" else NSAMPLE)
    out = {"workload": name, "params": {k: w[k] for k in ("lam", "theta", "order", "outer", "iters")},
           "sample_seed": 7, "indices": idx.tolist()}
    if name == "blobs96":
        loss, gm, gl = O.ssd_one_warping_grad(pair.fixed, pair.moving, w["lam"], w["theta"],
                                              w["order"], w["iters"])
        # probes: the voxel of largest |dL/dI1| in each 8^3 block, then the 16
        # blocks whose maxima are largest
        nz, ny, nx = gm.shape
        blk = np.abs(gm).reshape(nz // 8, 8, ny // 8, 8, nx // 8, 8).transpose(0, 2, 4, 1, 3, 5)
        blk = blk.reshape(nz // 8, ny // 8, nx // 8, 512)
        arg = blk.argmax(axis=-1)
        best = blk.max(axis=-1).reshape(-1)
        fd_idx = []
        for b in np.argsort(-best, kind="stable")[:16]:
            bz, by, bx = np.unravel_index(b, (nz // 8, ny // 8, nx // 8))
            iz, iy, ix = np.unravel_index(arg[bz, by, bx], (8, 8, 8))
            fd_idx.append(((bz * 8 + iz) * ny + by * 8 + iy) * nx + bx * 8 + ix)
        fd_idx = np.sort(np.array(fd_idx))
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
        r32 = oracle_register(w, pair.fixed, pair.moving)
        nb32 = nbhd_min_det(r32.disp).reshape(-1)
        near = np.setdiff1d(np.flatnonzero(nb32 <= FOLD_DET), idx)
        rng = np.random.default_rng(8)
        idx = np.sort(np.concatenate([idx, rng.choice(near, size=min(NFOLD_192, len(near)), replace=False)]))
        out["indices"] = idx.tolist()
        out["fold_samples"] = {"count": int(min(NFOLD_192, len(near))), "seed": 8, "nbhd_det_at_most": FOLD_DET}
        rb = oracle_register(w, synth.bf16_to_f32(fb), synth.bf16_to_f32(mb))
        out["bf16"] = run(w, synth.bf16_to_f32(fb), synth.bf16_to_f32(mb), idx, rb)
        out["fp32"] = run(w, pair.fixed, pair.moving, idx, r32)
        nbb = nbhd_min_det(rb.disp).reshape(-1)
        out["nbhd_min_det"] = {"fp32": [float(f"{v:.6g}") for v in nb32[idx]],
                               "bf16": [float(f"{v:.6g}") for v in nbb[idx]]}
        # what float32 arithmetic alone does: the oracle's steps in float32
        # against the FP64 oracle, over every voxel
        import fp32_mirror
        out["fp32_mirror"] = {}
        for key, (fi, mi), ref, nb in (("fp32", (pair.fixed, pair.moving), r32, nb32),
                                       ("bf16", (synth.bf16_to_f32(fb), synth.bf16_to_f32(mb)), rb, nbb)):
            md, mw = fp32_mirror.register_fp32(fi, mi, w["lam"], w["theta"], w["order"], w["outer"], w["iters"])
            de = np.abs(md.astype(np.float64) - ref.disp).max(axis=0).reshape(-1)
            we = np.abs(mw.astype(np.float64) - ref.warped).reshape(-1)
            away = nb > FOLD_DET
            out["fp32_mirror"][key] = {
                "disp_err_max": float(de.max()), "disp_err_mean": float(de.mean()),
                "warped_err_max": float(we.max()), "warped_err_mean": float(we.mean()),
                "voxels_beyond_1e-3_voxel_or_1e-4_intensity": int(((de > 1e-3) | (we > 1e-4)).sum()),
                "voxels_away_from_folds": int(away.sum()),
                "disp_err_max_away_from_folds": float(de[away].max()),
                "warped_err_max_away_from_folds": float(we[away].max())}
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
