#!/usr/bin/env python3
"""Benchmark: registrations/s and ms per ADMM iteration of the HIP path.

One step = one full registration (every stage of the path) of the 128x128x96
nested-ellipsoid heart phantom pair, 10 warpings x 20 Nesterov-ADMM
iterations, n = 2, lambda = 0.01, theta = 0.1, with inputs already resident
in GPU memory.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

HBM traffic of the dominant kernel comes from two rocprofv3 --pmc runs of
this script (FETCH_SIZE, then WRITE_SIZE) with --copy-probe, which first runs
a device-to-device copy of known size whose counter readings calibrate the
scale; `--traffic-from FETCH_CSV WRITE_CSV` turns the two counter files into
the record kept under profiles/.  The record names the digest of the kernel
sources it was taken on, and the bench line reports it only while the
sources still have that digest.
"""
from __future__ import annotations

import argparse
import csv
import math
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, packed (two lanes per instruction)
# Without packed FP32 instructions (disabled for every kernel here) one wave64
# FP32 FMA takes 4 cycles on a SIMD: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
FP32_NONPACKED_PEAK_TFLOPS = 78.6
# Compulsory bytes of one ADMM iteration (read w, w_old, b, b_old, J, r; write
# w, b: 22 float32 values per voxel), the unit the iteration rate is priced in.
ITER_FLOOR_BYTES_PER_VOXEL = 88.0
KERNEL_SOURCES = ["kernels.hip", "kernels.h", "fft_lds.h", "pointwise.h"]
# rocprofv3 kernel-name prefixes of the replayable kernels
KERNEL_NAMES = {"pass_a_fwd_x": "nadmm::k_pass_a<", "pass_b_yz_solve": "nadmm::k_pass_b<",
                "pass_ca_iter": "nadmm::k_pass_c<5,"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"

# Algorithmic bytes per voxel of each kernel kind (inputs read once, outputs
# written once; float32 fields, packed half spectrum = 4 B per component).
BYTES_PER_VOXEL = {
    # the registration's first pass of a warping (k_pass_a0, timed as pass_a_fwd_x):
    # I^w 4 + I0 4, write r 4 + s^0 12 + half spectrum 12; k_pass_a alone
    # (nadmm_admm, the replay) reads s^0 12 and writes the spectrum 12
    "pass_a_fwd_x": 36.0,
    "pass_b_yz_solve": 24.0,     # read + write the 3-component half spectrum
    "pass_ca_iter": 68.0,        # spectrum 12 + s^k, s^{k-1} 24 + I1^w 4 + r 4, write s 12 + spectrum 12
    "pass_c_compose": 44.0,      # spectrum 12 + u gather 12 + image gather 4, write u 12 + I^w 4
    "grad_resid": 24.0,          # I^w 4 + I0 4, write r 4 + s^0 12 (nadmm_warp and the gradient path)
    "warp": 20.0,                # u 12 + image 4, write 4
    "fill": 12.0,
}


def pass_b_flops(dims) -> float:
    """Nominal work of one y-z pass launch: per (component, x-frequency)
    plane of N = ny nz points a forward and an inverse 2-D FFT at
    5 N log2 N flops each, and the multiplier (~9 flops per point)."""
    nx, ny, nz = dims
    n = ny * nz
    return 3 * (nx // 2 + 1) * (2 * 5 * n * math.log2(n) + 9 * n)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="phantom128x128x96")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch of 32 uneven pairs (batched vs one-by-one)")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the gradient of one warping at 96^3")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the bfloat16-image run at 192x192x128 (vs the float32 path)")
    ap.add_argument("--no-threshold", action="store_true",
                    help="skip the threshold-stopped registration of the same pair")
    ap.add_argument("--no-pyramid", action="store_true",
                    help="skip the paper's three-level schedule on the same pair")
    ap.add_argument("--no-dram-check", action="store_true",
                    help="skip the 8-copy batched registration (the iteration beyond the Infinity Cache)")
    ap.add_argument("--shapes", type=lambda t: [int(v) for v in t.split(",")], default=None,
                    metavar="ROWS,COMPOSE_ROWS,PLANE_THREADS",
                    help="pin the launch shapes of the timed workload instead of autotuning them")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a device-to-device copy of known size first (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the traffic record from two rocprofv3 --pmc counter files and exit")
    args = ap.parse_args()
    if args.shapes is not None and len(args.shapes) != 3:
        ap.error("--shapes takes three integers: ROWS,COMPOSE_ROWS,PLANE_THREADS")
    return args


def sources_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2109_12688_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def copy_probe_bytes(V: int) -> int:
    return 3 * V * 4  # one vector field, read once and written once


def traffic_record(fetch_csv, write_csv, workload, kernel, shapes=None):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of `kernel`, each scaled by
    what the same counter reads for the copy probe of known size.  shapes:
    the launch shapes the profiled run was pinned to (--shapes), recorded
    with the workgroup size its dispatches had."""
    import numpy as np
    wg = {}

    def per_dispatch(path, counter):
        sums = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].replace("void ", "")
            key = next((k for k, pre in list(KERNEL_NAMES.items()) + [("copy", COPY_KERNEL)]
                        if name.startswith(pre)), None)
            if key is None:
                continue
            wg[key] = int(r["Workgroup_Size"])
            d = sums.setdefault(key, {})
            d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        # median over dispatches: the probe's copy kernel also serves a few
        # small runtime copies, and a warping's first iteration reads less
        return {k: float(np.median(list(v.values()))) for k, v in sums.items()}

    import synth
    V = int(np.prod(synth.WORKLOADS[workload]["dims"]))
    cb = copy_probe_bytes(V)
    f, w = per_dispatch(fetch_csv, "FETCH_SIZE"), per_dispatch(write_csv, "WRITE_SIZE")
    sf, sw = cb / (1024.0 * f["copy"]), cb / (1024.0 * w["copy"])
    rec = {"kernel": kernel, "workload": workload, "sources_sha256": sources_digest(),
           "fetch_kib_per_dispatch": round(f[kernel], 1), "write_kib_per_dispatch": round(w[kernel], 1),
           "copy_bytes": cb, "copy_fetch_kib": round(f["copy"], 1), "copy_write_kib": round(w["copy"], 1),
           "fetch_scale": round(sf, 4), "write_scale": round(sw, 4)}
    rec["read_bytes_per_launch"] = round(1024.0 * f[kernel] * sf)
    rec["write_bytes_per_launch"] = round(1024.0 * w[kernel] * sw)
    rec["traffic_bytes_per_launch"] = rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    rec["workgroup_size"] = wg.get(kernel)
    if shapes:
        rec["shapes"] = {"xline_rows": shapes[0], "compose_rows": shapes[1], "plane_threads": shapes[2]}
    return rec


def stored_traffic(workload, kernel, shapes=None):
    """HBM bytes per launch from the committed counter record, or None when
    there is none, the kernel sources changed since it was taken, or the
    record was taken at other x-line rows than `shapes` (tuned_shapes) has
    (the rows set which halo rows the fused pass re-reads)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("record: "):
            rec = json.loads(line[len("record: "):])
            if rec.get("sources_sha256") != sources_digest() or rec.get("kernel") != kernel:
                return None
            rs = rec.get("shapes")
            if shapes and rs and kernel == "pass_ca_iter" and rs["xline_rows"] != shapes["xline_rows"]:
                return None
            return rec
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(pair, w, extra=None):
    """The FP64 oracle on a bounded sample: the first half of the
    registration's warpings (each: warp of the moving image by the current
    displacement, gradient, `iters` ADMM iterations, composition) of the same
    workload, scaled to registrations/s."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O

    fixed = pair.fixed.astype(np.float64)
    moving = pair.moving.astype(np.float64)
    u = np.zeros((3,) + fixed.shape)
    n_w = max(1, w["outer"] // 2)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(n_w):
            _, J, r = O.warp_grad_residual(moving, fixed, u)
            res = O.admm(J, r, w["lam"], w["theta"], w["order"], w["iters"])
            u = O.compose(u, res.w)
        dt = time.perf_counter() - t0
    out = {"value": n_w / (w["outer"] * dt), "unit": "registrations/s", "cores": 1, "kind": "oracle",
           "sample": f"{n_w} of the {w['outer']} warpings ({w['iters']} ADMM iterations + warp + compose each), "
                     f"numpy float64 single thread, {dt:.2f} s"}
    out["s_per_admm_iter"] = round(dt / (n_w * w["iters"]), 4)
    out["others"] = cpu_others(extra or {})
    return out


def cpu_others(pairs):
    """The oracle, single-threaded, on the other workloads' bounded samples:
    the whole 32^3 blob registration (5 warpings x 10 iterations), and three
    ADMM iterations of the 192 x 192 x 128 phantom (per iteration)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    import synth

    res = {}
    with threadpool_limits(limits=1):
        wb = synth.WORKLOADS["blobs32"]
        pb = synth.make_pair("blobs32")
        t0 = time.perf_counter()
        O.register(pb.fixed.astype(np.float64), pb.moving.astype(np.float64), wb["lam"], wb["theta"],
                   wb["order"], wb["outer"], wb["iters"])
        dt = time.perf_counter() - t0
        res["blobs32"] = {"s_per_registration": round(dt, 3),
                          "s_per_admm_iter": round(dt / (wb["outer"] * wb["iters"]), 5)}
        if "phantom192x192x128" in pairs:
            p, w2 = pairs["phantom192x192x128"], synth.WORKLOADS["phantom192x192x128"]
            _, J, r = O.warp_grad_residual(p.moving.astype(np.float64), p.fixed.astype(np.float64),
                                           np.zeros((3,) + p.fixed.shape))
            t0 = time.perf_counter()
            O.admm(J, r, w2["lam"], w2["theta"], w2["order"], 3)
            res["phantom192x192x128"] = {"s_per_admm_iter": round((time.perf_counter() - t0) / 3, 4)}
    return res


def generate_inputs(args):
    """Every input pair, made in a process pool (the generators are pure NumPy
    on the host).  Runs before anything touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import synth

    jobs = {"main": (synth.make_pair, args.workload)}
    if not args.no_bf16:
        jobs["bf16"] = (synth.make_pair, "phantom192x192x128")
    if not args.no_grad:
        jobs["grad"] = (synth.make_pair, "blobs96")
    if not args.no_batch:
        for i, spec in enumerate(synth.batch_specs(32)):
            jobs[("batch", i)] = (synth.batch_pair, spec)
    workers = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    log(f"generating {len(jobs)} input pairs on {workers} processes")
    t0 = time.perf_counter()
    # fork (nothing has touched the GPU yet): spawn would leave its resource
    # tracker process running until the benchmark exits
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        futs = {k: ex.submit(f, a) for k, (f, a) in jobs.items()}
        out = {k: f.result() for k, f in futs.items()}
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")
    return out


def batch_vs_plain(api, torch, synth, pairs, reps=2):
    """The 32 uneven pairs registered one call per pair; batched per size (one
    nadmm_register_batch call per size, the three sizes on separate streams,
    eagerly and replayed from graphs); and in one nadmm_register_mixed call
    (one launch per phase over every pair of every size, eagerly and replayed
    from a graph).  Wall time of the whole set from HIP events on the
    launching stream; every pair checked bit for bit against its own call."""
    import numpy as np
    w = synth.BATCH_PARAMS
    specs = synth.batch_specs(32)
    args = (w["lam"], w["theta"], w["order"], w["outer"], w["iters"])
    single = [(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()) for f, m in pairs]
    sizes = sorted({d for d, _ in specs})
    ws1 = {d: api.workspace((d[2], d[1], d[0])) for d in sizes}
    outs = [None] * len(specs)

    def plain():
        for i, ((f, m), (d, _)) in enumerate(zip(single, specs)):
            outs[i] = api.register(f, m, *args, ws=ws1[d])

    groups = {}
    for i, (d, _) in enumerate(specs):
        groups.setdefault(d, []).append(i)
    stacked = {d: (torch.stack([single[i][0] for i in idx]), torch.stack([single[i][1] for i in idx]))
               for d, idx in groups.items()}
    wsb = {d: api.workspace_batch((d[2], d[1], d[0]), len(idx)) for d, idx in groups.items()}
    streams = {d: torch.cuda.Stream() for d in groups}
    bouts = {}
    for d, idx in groups.items():
        api.autotune((d[2], d[1], d[0]), w["lam"], w["theta"], w["order"], batch=len(idx), ws=wsb[d])
    tiles = {"x".join(map(str, d)): api.tuned_shapes((d[2], d[1], d[0])) for d in groups}

    def batched():
        cur = torch.cuda.current_stream()
        for d in groups:
            s = streams[d]
            s.wait_stream(cur)
            with torch.cuda.stream(s):
                bouts[d] = api.register_batch(stacked[d][0], stacked[d][1], *args, ws=wsb[d])
        for d in groups:
            cur.wait_stream(streams[d])

    def ms(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cur = torch.cuda.current_stream()
        e0.record(cur)
        for _ in range(reps):
            fn()
        e1.record(cur)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_plain = ms(plain)
    t_batch = ms(batched)
    # the batched set captured once in a graph per size class (launch work
    # recorded, replayed on the same streams)
    graphs = {}
    for d in groups:
        s = streams[d]
        s.wait_stream(torch.cuda.current_stream())
        graphs[d] = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graphs[d], stream=s):
            api.register_batch(stacked[d][0], stacked[d][1], *args, ws=wsb[d], out=bouts[d])
    torch.cuda.synchronize()

    def batched_graph():
        cur = torch.cuda.current_stream()
        for d in groups:
            s = streams[d]
            s.wait_stream(cur)
            with torch.cuda.stream(s):
                graphs[d].replay()
        for d in groups:
            cur.wait_stream(streams[d])

    t_graph = ms(batched_graph)
    same = all(torch.equal(bouts[d]["disp"][j], outs[i]["disp"]) for d, idx in groups.items()
               for j, i in enumerate(idx))  # after the graph replays

    # all 32 pairs in one call, one launch per phase over every size
    # (nadmm_register_mixed), eagerly and replayed from a graph
    fl, ml = [f for f, _ in single], [m for _, m in single]
    wsm = api.workspace_mixed([tuple(f.shape) for f in fl])
    mixed_out = api.register_mixed(fl, ml, *args, ws=wsm)
    packed = mixed_out["packed"]
    t_mixed = ms(lambda: api.register_mixed(fl, ml, *args, ws=wsm, packed=packed))
    same_mixed = all(torch.equal(mixed_out["disp"][i], outs[i]["disp"]) and
                     torch.equal(mixed_out["warped"][i], outs[i]["warped"]) for i in range(len(specs)))
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    gm = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gm, stream=gs):
        api.register_mixed(fl, ml, *args, ws=wsm, packed=packed)
    torch.cuda.synchronize()
    t_mixed_graph = ms(lambda: gm.replay())
    same_mixed = same_mixed and all(torch.equal(mixed_out["disp"][i], outs[i]["disp"]) for i in range(len(specs)))
    log(f"batch of {len(specs)}: one call over all sizes {t_mixed:.2f} ms, replayed graph {t_mixed_graph:.2f} ms")
    nvox = int(sum(np.prod(d) for d, _ in specs))
    log(f"batch of {len(specs)}: one by one {t_plain:.2f} ms, batched {t_batch:.2f} ms")
    return {"pairs": len(specs), "sizes": {"x".join(map(str, d)): len(idx) for d, idx in groups.items()},
            "voxels": nvox, "outer": w["outer"], "iters": w["iters"], "steps": reps,
            "ms_one_by_one": round(t_plain, 3), "ms_batched": round(t_batch, 3),
            "ms_batched_graph": round(t_graph, 3),
            "pairs_per_s_one_by_one": round(1000.0 * len(specs) / t_plain, 2),
            "pairs_per_s_batched": round(1000.0 * len(specs) / t_batch, 2),
            "batched_vs_one_by_one": round(t_plain / t_batch, 4),
            "batched_graph_vs_one_by_one": round(t_plain / t_graph, 4),
            "ms_mixed_one_call": round(t_mixed, 3), "ms_mixed_graph": round(t_mixed_graph, 3),
            "pairs_per_s_mixed": round(1000.0 * len(specs) / t_mixed, 2),
            "mixed_vs_one_by_one": round(t_plain / t_mixed, 4),
            "mixed_vs_per_size_streams": round(t_batch / t_mixed, 4),
            "tuned_shapes": tiles,
            "bit_identical": bool(same), "mixed_bit_identical": bool(same_mixed)}


# The paper's runtime per pair for the L2 data term with the second-order
# regulariser (Table 1, NVIDIA V100, first hyper-parameter version): context
# for the same schedule below, not a target (other hardware, other images).
PAPER_V1_SECONDS = 1.38
# ... and of its second version (threshold stopping), same table.
PAPER_V2_SECONDS = 5.00


def pyramid_time(api, torch, pair, w, reps=5):
    """The paper's first hyper-parameter schedule on the same phantom pair:
    three levels, coarsest first, 10 / 10 / 5 warpings of 10 / 5 / 5 ADMM
    iterations (nadmm_register_pyramid): ms per registration."""
    f, m = torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda()
    outer, iters = (10, 10, 5), (10, 5, 5)
    ws = api.workspace_pyramid(pair.fixed.shape, outer, iters)
    stream = torch.cuda.current_stream()
    run = lambda: api.register_pyramid(f, m, w["lam"], w["theta"], w["order"], outer, iters, ws=ws)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps
    log(f"pyramid (paper's first schedule): {t:.3f} ms per registration")
    res = {"levels": 3, "warpings": list(outer), "iters": list(iters), "order": "coarsest first",
           "steps": reps, "ms_per_registration": round(t, 3),
           "paper_v100_seconds_context": PAPER_V1_SECONDS}
    # the paper's second version: the same pyramid with threshold stopping
    # (ADMM 0.05 within its 0.01 .. 0.13, warpings 2 %), caps 20 x 40 per level
    outer2, iters2, ta, tw = (20, 20, 20), (40, 40, 40), 0.05, 0.02
    ws2 = api.workspace_pyramid(pair.fixed.shape, outer2, iters2)
    run2 = lambda: api.register_pyramid_threshold(f, m, w["lam"], w["theta"], w["order"], outer2, iters2, ta, tw,
                                                  ws=ws2)
    out = run2()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = run2()
    t2 = (time.perf_counter() - t0) / reps * 1e3
    its = out["level_iters"]
    log(f"pyramid with threshold stopping: {t2:.3f} ms per registration, warpings {out['outer_run']}, "
        f"ADMM iterations {[sum(x) for x in its]}")
    res["threshold"] = {"tol_admm": ta, "tol_warp": tw, "cap_warpings": list(outer2), "cap_iters": list(iters2),
                        "ms_per_registration": round(t2, 3), "warpings": out["outer_run"],
                        "admm_iterations": [sum(x) for x in its],
                        "paper_v100_seconds_context": PAPER_V2_SECONDS}
    return res


def threshold_time(api, torch, pair, w, reps=3):
    """Threshold stopping (nadmm_register_threshold) on the same phantom pair:
    the ADMM loop stops at a relative change of its w-step input below
    0.05 (the paper's thresholds range over 0.01 .. 0.13), the warping loop
    at a displacement change below 2 %; caps 10 warpings x 40 iterations.
    The call is synchronous (one read-back per check): wall clock."""
    f, m = torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda()
    ws = api.workspace(pair.fixed.shape)
    outer, iters, ta, tw = 10, 40, 0.05, 0.02
    run = lambda: api.register_threshold(f, m, w["lam"], w["theta"], w["order"], outer, iters, ta, tw, ws=ws)
    res = run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = run()
    t = (time.perf_counter() - t0) / reps * 1e3
    n_it = sum(res["iters_run"])
    checks = sum(len(c) for c in res["admm_change"]) + len(res["warp_change"])
    log(f"threshold stopping: {t:.3f} ms per registration, {res['outer_run']} warpings, "
        f"{n_it} ADMM iterations, {checks} checks")
    return {"tol_admm": ta, "tol_warp": tw, "cap_warpings": outer, "cap_iters": iters, "steps": reps,
            "ms_per_registration": round(t, 3), "warpings": res["outer_run"], "iters_run": res["iters_run"],
            "admm_iterations": n_it, "checks": checks, "ms_per_admm_iter": round(t / n_it, 5)}


def grad_time(api, torch, synth, pair, reps=5):
    """The differentiated warping at 96^3 (20 iterations, checkpoints every
    5): ms per call of the gradient entry point (loss, dL/dmoving,
    dL/dlambda), against one forward warping (nadmm_register, 1 x 20)."""
    name = "blobs96"
    w = synth.WORKLOADS[name]
    f, m = torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda()
    args = (w["lam"], w["theta"], w["order"], w["iters"])
    ws = api.workspace_grad(pair.fixed.shape, *args, w["checkpoint"])
    wsr = api.workspace(pair.fixed.shape)
    stream = torch.cuda.current_stream()

    def ms(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_grad = ms(lambda: api.ssd_grad(f, m, *args, checkpoint=w["checkpoint"], ws=ws))
    t_fwd = ms(lambda: api.register(f, m, w["lam"], w["theta"], w["order"], 1, w["iters"], ws=wsr))
    log(f"{name}: gradient {t_grad:.3f} ms, forward warping {t_fwd:.3f} ms")
    return {"workload": name, "dims_xyz": list(w["dims"]), "iters": w["iters"],
            "checkpoint": w["checkpoint"], "steps": reps, "ms_per_gradient": round(t_grad, 3),
            "ms_per_forward_warping": round(t_fwd, 3), "gradient_vs_forward": round(t_grad / t_fwd, 3)}


def sample_errors(res, golden, key):
    """Per-output errors of one registration against the FP64 oracle's
    stored samples (tests/golden/, written by make_golden.py from the oracle
    only): displacement (max over components), warped intensity, and both
    restricted to the samples whose oracle determinant stays above 0.1 in the
    9^3 neighbourhood (away from folds)."""
    import numpy as np
    idx = np.array(golden["indices"])
    g = golden[key]
    disp = res["disp"].reshape(3, -1)[:, idx].double().cpu().numpy()
    warped = res["warped"].reshape(-1)[idx].double().cpu().numpy()
    de = np.abs(disp - np.array(g["disp"])).max(axis=0)
    we = np.abs(warped - np.array(g["warped"]))
    away = np.array(golden["nbhd_min_det"][key]) > 0.1
    return {"samples": int(len(idx)), "disp_err_max": float(de.max()), "disp_err_mean": float(de.mean()),
            "warped_err_max": float(we.max()), "warped_err_mean": float(we.mean()),
            "samples_beyond_1e-3_voxel_or_1e-4_intensity": int(((de > 1e-3) | (we > 1e-4)).sum()),
            "samples_away_from_folds": int(away.sum()),
            "disp_err_max_away_from_folds": float(de[away].max()),
            "warped_err_max_away_from_folds": float(we[away].max()),
            "oracle_min_det_J": g["jacobian"]["min"], "oracle_n_det_nonpos": g["jacobian"]["n_nonpos"]}


def dram_check(api, torch, pair, w, single_iter_ms, reps=3, copies=8):
    """The headline iteration with a working set far beyond the 256 MB
    Infinity Cache: `copies` copies of the same pair in one batched call
    (one launch per phase covers all of them), the ADMM iteration time per
    pair from the difference of two iteration counts as for the headline
    figure.  About 70 MB per pair per iteration, 560 MB for 8 pairs: what
    this rate loses against the single pair's is what the Infinity Cache
    was adding."""
    import numpy as np
    shp = pair.fixed.shape
    f = torch.from_numpy(np.stack([pair.fixed] * copies)).cuda()
    m = torch.from_numpy(np.stack([pair.moving] * copies)).cuda()
    ws = api.workspace_batch(shp, copies)
    out = None
    stream = torch.cuda.current_stream()

    def ms(iters):
        nonlocal out
        run = lambda: api.register_batch(f, m, w["lam"], w["theta"], w["order"], w["outer"], iters, ws=ws,
                                          out=out)
        out = run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    half = w["iters"] // 2
    t_full, t_half = ms(w["iters"]), ms(half)
    it_ms = (t_full - t_half) / (w["outer"] * (w["iters"] - half) * copies)
    V = int(np.prod(shp))
    ach = ITER_FLOOR_BYTES_PER_VOXEL * V / (it_ms * 1e-3) / 1e9
    log(f"{copies} copies batched: {t_full / copies:.3f} ms per pair, {1e3 * it_ms:.2f} us per pair-iteration")
    nz, ny, nx = shp
    per_pair = 32 * V + 24 * (nx // 2 + 1) * ny * nz  # s^k, s^(k-1), I1^w, r and the half spectrum
    return {"pairs": copies, "working_set_mb_per_iteration": round(copies * per_pair / 1e6, 1),
            "ms_per_registration_per_pair": round(t_full / copies, 4),
            "ms_per_admm_iter_per_pair": round(it_ms, 5),
            "iteration_achieved_gbs": round(ach, 1), "iteration_frac": round(ach / HBM_PEAK_GBS, 4),
            "vs_single_pair_iteration": round(single_iter_ms / it_ms, 4)}


def bf16_vs_plain(api, torch, synth, pair, reps=3):
    """The precision workload (192x192x128 phantom, n = 3, lambda = 0.005,
    10 x 30) registered from bfloat16 and from float32 images on the same
    GPU: ms per registration of each (event-timed, inputs resident), each
    output's error against the FP64 oracle's stored samples, and the ADMM
    iteration's roofline at this size (a working set larger than the
    256 MB Infinity Cache)."""
    name = "phantom192x192x128"
    w = synth.WORKLOADS[name]
    shp = pair.fixed.shape
    ws = api.workspace(shp)
    f32 = (torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda())
    b16 = tuple(t.to(torch.bfloat16) for t in f32)
    out = {"disp": torch.empty((3,) + shp, device="cuda"), "warped": torch.empty(shp, device="cuda")}
    stream = torch.cuda.current_stream()

    def run(imgs):
        return api.register(imgs[0], imgs[1], w["lam"], w["theta"], w["order"], w["outer"], w["iters"],
                            ws=ws, out=out)

    def ms(imgs):
        run(imgs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run(imgs)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    with open(os.path.join(ROOT, "tests", "golden", f"{name}_oracle_samples.json")) as f:
        golden = json.load(f)
    plain = ms(f32)
    torch.cuda.synchronize()
    err_fp32 = sample_errors(out, golden, "fp32")
    bf = ms(b16)
    torch.cuda.synchronize()
    err_bf16 = sample_errors(out, golden, "bf16")
    stats, nneg, _ = api.jacobian(out["disp"], ws=ws)
    torch.cuda.synchronize()
    err_bf16.update({"min_det_J": float(stats[0].item()), "n_det_nonpos": int(nneg.item())})
    run(f32)
    stats, nneg, _ = api.jacobian(out["disp"], ws=ws)
    torch.cuda.synchronize()
    err_fp32.update({"min_det_J": float(stats[0].item()), "n_det_nonpos": int(nneg.item())})
    log(f"{name}: float32 images {plain:.3f} ms, bfloat16 images {bf:.3f} ms per registration")
    log(f"{name}: errors vs oracle samples, float32 images {err_fp32}, bfloat16 images {err_bf16}")
    rl = iteration_rooflines(api, lambda: run(f32), shp, w, ws, name, reps=50)
    return {"workload": name, "dims_xyz": list(w["dims"]), "outer": w["outer"], "iters": w["iters"],
            "order": w["order"], "lambda": w["lam"], "steps": reps,
            "ms_per_registration_fp32_images": round(plain, 3),
            "ms_per_registration_bf16_images": round(bf, 3),
            "registrations_per_s_bf16": round(1000.0 / bf, 3),
            "bf16_vs_plain": round(plain / bf, 4),
            "errors_vs_oracle": {"fp32_images": err_fp32, "bf16_images": err_bf16},
            "rooflines": rl}


def iteration_rooflines(api, step, shp, w, ws, workload, reps=200):
    """Rooflines of the ADMM iteration, measured by replaying its kernels on
    the state a registration left in the workspace (nadmm_profile_replay:
    `reps` launches back to back between two HIP events on the launch
    stream, so launch gaps are included).

    admm_iteration: the unit of the iteration rate, priced at its compulsory
    88 B/voxel against the HBM peak (the two launches move 92 B/voxel).
    pass_ca_iter: the fused x-line pass, HBM-bound, at its own 68 B/voxel.
    pass_b_yz_solve: the y-z spectral pass at its 24 B/voxel against HBM, and
    its nominal FFT work against the non-packed FP32 vector rate."""
    import numpy as np
    V = int(np.prod(shp))
    shapes = api.tuned_shapes(shp)
    out = {}
    for kind in ("admm_iteration", "pass_ca_iter", "pass_b_yz_solve"):
        step()
        avg_s = api.profile_replay(shp, kind, reps, w["lam"], w["theta"], w["order"], ws) / 1e3
        if kind == "admm_iteration":
            bpl = ITER_FLOOR_BYTES_PER_VOXEL * V
            tr = [stored_traffic(workload, k, shapes) for k in ("pass_ca_iter", "pass_b_yz_solve")]
            traffic = (sum(t["traffic_bytes_per_launch"] for t in tr) if all(tr) else None)
        else:
            bpl = BYTES_PER_VOXEL[kind] * V
            t = stored_traffic(workload, kind, shapes)
            traffic = t["traffic_bytes_per_launch"] if t else None
        ach = bpl / avg_s / 1e9
        r = {"kernel": kind, "avg_us": round(avg_s * 1e6, 3), "bytes_per_launch": bpl, "bound": "hbm",
             "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic}
        if kind == "admm_iteration":
            r["kernel"] = "admm_iteration (pass_ca_iter + pass_b_yz_solve)"
            r["bytes_per_voxel"] = ITER_FLOOR_BYTES_PER_VOXEL
        if kind == "pass_b_yz_solve":
            fl = pass_b_flops(w["dims"])
            r["alu"] = {"achieved": round(fl / avg_s / 1e12, 2), "peak": FP32_NONPACKED_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(fl / avg_s / 1e12 / FP32_NONPACKED_PEAK_TFLOPS, 4),
                        "flops_per_launch": round(fl)}
        out[kind] = r
    return out


def main():
    args = parse()
    if args.traffic_from:
        for kind in ("pass_ca_iter", "pass_b_yz_solve"):
            print("record: " + json.dumps(traffic_record(args.traffic_from[0], args.traffic_from[1],
                                                           args.workload, kind, args.shapes)))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): registrations would shard "
              "by pair over several GPUs, which this benchmark does not run", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    inputs = generate_inputs(args)  # before any GPU use
    import torch

    import synth
    from paper_2109_12688_amd import _lib, api

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    pair = inputs["main"]
    fixed = torch.from_numpy(pair.fixed).cuda()
    moving = torch.from_numpy(pair.moving).cuda()
    shp = tuple(fixed.shape)
    V = int(np.prod(shp))
    ws = api.workspace(shp)
    out = {"disp": torch.empty((3,) + shp, device="cuda"), "warped": torch.empty(shp, device="cuda")}

    def step():
        return api.register(fixed, moving, w["lam"], w["theta"], w["order"], w["outer"], w["iters"],
                            ws=ws, out=out)

    stream = torch.cuda.current_stream()
    # achievable copy bandwidth (device-to-device copy of one vector field)
    src = torch.rand((3,) + shp, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3 if args.copy_probe else 1):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ncopy = 50
    c0.record(stream)
    for _ in range(ncopy):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * copy_probe_bytes(V) / (c0.elapsed_time(c1) / ncopy * 1e-3) / 1e9
    del src, dst

    if args.shapes:
        # pinned shapes (profiled runs: a profiler distorts the autotuner's timings)
        api.set_shapes(shp, *args.shapes)
    else:
        api.autotune(shp, w["lam"], w["theta"], w["order"], ws=ws)
    shapes = api.tuned_shapes(shp)
    log(f"tuned shapes: {shapes}")
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    log(f"timing {args.steps} registrations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev[0].elapsed_time(ev[-1]) / args.steps
    per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    log(f"{ms_per_step:.3f} ms/registration (wall {1e3 * wall / args.steps:.3f})")

    # ms per ADMM iteration as the inner-loop time over outer x iters: the
    # same registration at `iters` and at iters / 2 iterations per warping
    # differ by exactly outer x (iters - iters / 2) iterations (a warping's
    # first iteration, its composition and the warp are in both)
    half = w["iters"] // 2

    def reg_ms(iters, reps):
        run = lambda: api.register(fixed, moving, w["lam"], w["theta"], w["order"], w["outer"], iters,
                                   ws=ws, out=out)
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_full, t_half = reg_ms(w["iters"], args.steps), reg_ms(half, args.steps)
    ms_per_iter = (t_full - t_half) / (w["outer"] * (w["iters"] - half))
    log(f"ms per ADMM iteration: ({t_full:.3f} - {t_half:.3f}) / ({w['outer']} x {w['iters'] - half})"
        f" = {ms_per_iter:.5f}")

    # per-kernel durations from HIP events bracketing each library launch
    # (each bracket adds the launch gap)
    _lib.profile_enable(True)
    for _ in range(args.profile_steps):
        step()
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    kernels = {}
    for k, (n, ms) in prof.items():
        kernels[k] = {"launches_per_step": n / args.profile_steps, "avg_us_event_bracketed": 1e3 * ms / n}
    rooflines = iteration_rooflines(api, step, shp, w, ws, args.workload)
    roofline = dict(rooflines["admm_iteration"])
    roofline["copy_gbs"] = round(copy_gbs, 1)
    roofline["ms_per_admm_iter_differenced"] = round(ms_per_iter, 5)

    stats, nneg, _ = api.jacobian(out["disp"], ws=ws)
    torch.cuda.synchronize()
    res = {
        "metric": "registrations/sec + ms per ADMM iter at 128x128x96; batched/BF16 vs plain",
        "value": round(1000.0 / ms_per_step, 3),
        "unit": "registrations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_p10_p50_p90": [round(float(np.percentile(per_step, q)), 4) for q in (10, 50, 90)],
        "ms_per_admm_iter": round(ms_per_iter, 5),
        "ms_per_admm_iter_method": (f"(registration at {w['iters']} iterations per warping - at {half}) / "
                                    f"({w['outer']} warpings x {w['iters'] - half})"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "inputs": ("seeded nested-ellipsoid heart phantom pair (stand-in for the paper's cardiac MRI); the random "
                   "deformation's exponential integrated by RK4 on a spline interpolant instead of the 6 "
                   "scaling-and-squaring steps the workload text names (the input generator carries none of "
                   "the method's arithmetic)"),
        "config": {"workload": args.workload, "dims_xyz": list(w["dims"]), "outer": w["outer"],
                   "iters": w["iters"], "order": w["order"], "lambda": w["lam"], "theta": w["theta"],
                   "parallelism": "single-gpu", "tuned_shapes": shapes},
        "roofline": roofline,
        "rooflines": rooflines,
        "kernels": kernels,
        "min_det_J": float(stats[0].item()),
        "n_det_nonpos": int(nneg.item()),
    }
    if not args.no_dram_check:
        res["dram_check"] = dram_check(api, torch, pair, w, ms_per_iter)
    if not args.no_bf16:
        res["bf16"] = bf16_vs_plain(api, torch, synth, inputs["bf16"])
    if not args.no_grad:
        res["grad"] = grad_time(api, torch, synth, inputs["grad"])
    if not args.no_pyramid:
        res["pyramid"] = pyramid_time(api, torch, pair, w)
    if not args.no_threshold:
        res["threshold"] = threshold_time(api, torch, pair, w)
    if not args.no_batch:
        res["batch"] = batch_vs_plain(api, torch, synth,
                                      [inputs[("batch", i)] for i in range(32)])
    if not args.no_cpu_baseline:
        log("timing the oracle sample on the CPU")
        res["cpu_baseline"] = cpu_baseline(pair, w, {"phantom192x192x128": inputs["bf16"]} if "bf16" in inputs
                                           else None)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
