"""Spin-image generation benchmark on one MI355X.

Main workload (seeded, synthetic): the clustered primitives scene --
2,000,000 float32 oriented points on 400 random tori and ellipsoids whose
centres are Gaussian-clustered (sigma 1) in a [0, 40]^3 box, per-object
density varying tenfold -- with every point oriented, W = 32, bin 0.02,
support angle 60 degrees, bilinear binning, FAC chunking on the persistent
kernel: factoring with ratio 16 and chunks of at least 32 images over the
contiguous cell order (MAIN_SCHED below), the autotuner's locality preset;
FAC2 on the spread order, the library's default, is timed beside it with the
other techniques.

One timed step = the whole hot path: si_build_scene (bounding box, cell
binning, scan, scatter) followed by si_generate (cell ordering, FAC chunk
claims, candidate culling, pair tests, LDS accumulation, image write-back),
inputs already resident in HBM.  The reported value is in-support point pairs
binned per second over the step; images per second beside it.

Also reported (outside the timed steps):
  * generation time of every schedule (STATIC, SS, GSS, FAC, LEARNED) with
    its speedup over STATIC and a bit-identity check of the images;
  * the learned cost model: trained on the in-support counts logged on the
    100k-point primitives scene and on this scene (80/20 split), held-out MAE;
  * the schedules under emulated heterogeneous workers (half the workgroups
    2x slower, idling or busy), and the claim-order effect of GSS;
  * next to the path: mesh resolution, normal estimation and spin-image
    matching (correlation on the matrix cores, against its roofline);
  * batching: 256 primitive scenes of log-uniform size in [1k, 200k] points
    and mixed W in {16, 32, 64}, one autotuned HIP-graph launch against a loop
    of 256 si_generate calls;
  * the roofline of the spin kernel and the FP64 CPU oracle timed on a
    bounded sample of the main workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-schedules] [--no-batch] [--no-extent] [--no-paper-shape]
                    [--no-adjacent] [--copy-calibration BYTES]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "in-support point-pairs binned/sec + spin-images/sec; learned vs FAC vs static"

# Algorithmic work per unit (VALU lane operations), counted on the definition
# rather than on executed instructions:
#   every in-extent pair (inside the beta/alpha window, whatever its angle):
#     3 subtractions, two 3-term dot products and a 3-term squared norm
#     (9 mul/fma), 1 fma for alpha^2, 4 comparisons          -> 17 ops
#   every in-support pair, bilinear: v, u (sqrt counted as 4), floors,
#     conversions, clamps, fractional parts, 16.16 weights    -> 26 ops
#     + 4 LDS atomic adds
OPS_PER_EXTENT_PAIR = 17
OPS_PER_SUPPORT_PAIR = 26
ATOMICS_PER_SUPPORT_PAIR = 4
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz non-packed FP32/INT VALU
# lane-operations per second (the 157.3 TFLOP/s figure counts an FMA as two
# flops and needs packed dual FP32, which the library's kernels do not use).
PEAK_VALU_OPS = 256 * 64 * 2.4e9


# HBM bytes per spin-kernel launch on the main workload, from two counter runs
# (FETCH_SIZE, WRITE_SIZE) calibrated on a plain copy; recorded with a hash of
# the kernel sources it was measured on and reported only while they match.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spin_clustered2m_traffic.json")

# The main step's schedule: factoring (FAC, Section 2.2) with ratio x = 16 and
# a minimum chunk of 32 images over the contiguous cell order.  Small chunks
# there make all workgroups sweep the scene together, so the candidates of
# the groups running at once share the L2; FAC's shrinking chunks keep the
# tail balanced.  The traffic record holds the schedule it was measured with.
MAIN_SCHED = {"kind": "fac", "fac_divisor": 16.0, "min_chunk": 32, "order": "cell"}
MAIN_SCHED_DESC = "FAC, ratio 16, minimum chunk 32, cell order, default group and workgroups"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1811_00901_amd", "csrc", f)
                  for f in ("k_spin.hip", "si_internal.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if rec.get("schedule") != MAIN_SCHED_DESC:
        return None
    return rec.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="clustered2m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-schedules", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-paper-shape", action="store_true")
    ap.add_argument("--no-adjacent", action="store_true",
                    help="skip mesh resolution, normal estimation and spin-image matching")
    ap.add_argument("--no-extent", action="store_true",
                    help="stop after the timed steps (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    # images of the paper-shaped loop in the host replica of the paper's
    # experiment (the oracle under STATIC, SS, GSS and FAC2; 0 = skip)
    ap.add_argument("--cpu-sched-images", type=int, default=4096)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, copy BYTES device-to-device once, so that a "
                         "counter run sees a plain copy of known size beside the spin kernel")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


WARM, REPS = 3, 15   # warm-ups and timed repetitions of every comparison


def spread(ts):
    """Median, quartiles and extremes of a list of times (ms)."""
    q = np.percentile(np.asarray(ts, dtype=np.float64), [0, 25, 50, 75, 100])
    return {"median": float(q[2]), "q1": float(q[1]), "q3": float(q[3]),
            "min": float(q[0]), "max": float(q[4])}


def timed(torch, fn, reps=REPS, warm=WARM):
    """Wall times (ms) of fn() between device synchronisations: spread()."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return spread(ts)


def train_cost_model(torch, si, sg, main):
    """Train the cost model on counts logged by the library on the 100k-point
    primitives scene and on the main scene; 80/20 split, seed 5."""
    cfg = sg.CONFIGS["prims100k"]
    xyz, nrm = sg.config_scene("prims100k")
    p2 = si.Params(cfg.W, cfg.bin, cfg.support_angle)
    sc2 = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(),
                            si.si_support_radius(p2))
    idx2 = torch.arange(cfg.N, dtype=torch.int32, device="cuda")
    _, cnt2, _ = si.si_generate(sc2, idx2, p2, si.Sched("fac"))
    feats = torch.cat([si.si_features(sc2, idx2, p2),
                       si.si_features(main["scene"], main["idx"], main["params"])])
    counts = torch.cat([cnt2, main["counts"]])
    n = int(feats.shape[0])
    perm = torch.from_numpy(np.random.default_rng(5).permutation(n)).cuda()
    n_tr = int(0.8 * n)
    f_tr, c_tr = feats[perm[:n_tr]].contiguous(), counts[perm[:n_tr]].contiguous()
    f_te, c_te = feats[perm[n_tr:]].contiguous(), counts[perm[n_tr:]].contiguous()
    y_te = c_te.to(torch.float64)
    model = si.si_cost_model_create(5)
    mae0 = float((si.si_cost_model_predict(model, f_te).double() - y_te).abs().mean())
    torch.cuda.synchronize()
    t = time.perf_counter()
    curve = si.si_cost_model_train(model, f_tr, c_tr, epochs=4, lr=2e-3, batch=4096)
    train_s = time.perf_counter() - t
    mae = float((si.si_cost_model_predict(model, f_te).double() - y_te).abs().mean())
    # baselines on the same held-out samples: the training mean, and the
    # occupancy sum (count proportional to the 27-cell candidate count,
    # feature 10 = log1p of it, the ratio fitted on the training samples)
    y_tr = c_tr.to(torch.float64)
    mae_mean = float((y_tr.mean() - y_te).abs().mean())
    occ_tr = torch.expm1(f_tr[:, 10].double())
    occ_te = torch.expm1(f_te[:, 10].double())
    mae_occ = float((y_tr.sum() / occ_tr.sum() * occ_te - y_te).abs().mean())
    info = {"samples_train": n_tr, "samples_test": n - n_tr, "epochs": 4, "batch": 4096,
            "lr": 2e-3, "train_s": train_s, "loss_curve": [float(x) for x in curve],
            "mae_test": mae, "mae_test_untrained": mae0, "mae_test_train_mean": mae_mean,
            "mae_test_occupancy_sum": mae_occ, "mean_count_test": float(y_te.mean()),
            "data": "counts logged on prims100k (65,536 images) + clustered2m (2,000,000 images)"}
    sc2.free()
    return model, info


def batched(torch, si, sg, model):
    """256 uneven scenes: a loop of si_generate calls against one batched
    graph launch (FAC with default and autotuned parameters, and LEARNED with
    the trained model on the tuned parameters); scene builds timed apart, one
    si_build_scene per scene and one si_build_scenes for all."""
    specs = sg.batch_specs(256)
    raw, items = [], []
    for seed, M, W in specs:
        xyz, nrm = sg.batch_scene(seed, M)
        params = si.Params(W, 0.02, float(np.float32(math.pi / 3)))
        raw.append((torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(),
                    si.si_support_radius(params)))
        idx = torch.arange(M, dtype=torch.int32, device="cuda")
        img = torch.empty((M, W, W), dtype=torch.float32, device="cuda")
        cnt = torch.empty((M,), dtype=torch.int32, device="cuda")
        items.append([None, idx, params, img, cnt])

    def build():
        scenes = [si.si_build_scene(x, n, r) for x, n, r in raw]
        for it, sc in zip(items, scenes):
            if it[0] is not None:
                it[0].free()
            it[0] = sc

    build_ms = timed(torch, build, reps=5, warm=1)

    def build_batched():
        scenes = si.si_build_scenes(raw)
        for it, sc in zip(items, scenes):
            if it[0] is not None:
                it[0].free()
            it[0] = sc

    build_batched_ms = timed(torch, build_batched, reps=5, warm=1)
    total_img = sum(int(it[1].shape[0]) for it in items)
    fac = si.Sched("fac")

    def loop():
        for scene, idx, params, img, cnt in items:
            si.si_generate(scene, idx, params, fac, img, cnt)

    loop_ms = timed(torch, loop)
    ref = [(img.clone(), cnt.clone()) for _, _, _, img, cnt in items]
    pairs = sum(int(c.to(torch.int64).sum()) for _, c in ref)
    tuned, _ = si.si_autotune(items, "fac", use_graph=True, max_trials=24)
    graph_ms = timed(torch, lambda: si.si_generate_batched(items, tuned, use_graph=True))
    default_ms = timed(torch, lambda: si.si_generate_batched(items, fac, use_graph=True))
    same = all(torch.equal(img, r[0]) and torch.equal(cnt, r[1])
               for (_, _, _, img, cnt), r in zip(items, ref))
    learned = None
    if model is not None:
        # the tuned launch shape (group, workgroups); its own chunk sizes and
        # order (FAC's tuned ratio and minimum chunk size FAC's chunks)
        ls = si.Sched("learned", tuned.num_workgroups, 0, 0.0, model, True, tuned.group)
        learned_ms = timed(torch, lambda: si.si_generate_batched(items, ls, use_graph=True))
        st = si.si_generate_batched(items, ls, use_graph=True, stats=True)
        # the same with the library's defaults (no tuning)
        ld = si.Sched("learned", model=model)
        learned_default_ms = timed(torch, lambda: si.si_generate_batched(items, ld, use_graph=True))
        learned = {"ms": learned_ms, "default_ms": learned_default_ms,
                   "speedup_default_vs_fac_default":
                       default_ms["median"] / learned_default_ms["median"],
                   "sched_used": list(si.SCHED)[st["sched_used"]],
                   "n_chunks": st["n_chunks"],
                   "identical": all(torch.equal(img, r[0]) and torch.equal(cnt, r[1])
                                    for (_, _, _, img, cnt), r in zip(items, ref)),
                   "speedup_vs_fac_tuned": graph_ms["median"] / learned_ms["median"]}
    best = min(graph_ms["median"], learned["ms"]["median"] if learned else float("inf"))
    out = {"workload": "256 primitive scenes, M log-uniform in [1k, 200k], W in {16,32,64}, "
                       "bin 0.02, 60 deg, all points oriented",
           "points": int(sum(s[1] for s in specs)), "images": total_img, "in_support_pairs": pairs,
           "build_ms": build_ms, "build_batched_ms": build_batched_ms,
           "loop_ms": loop_ms, "graph_default_ms": default_ms,
           "graph_tuned_ms": graph_ms, "graph_learned": learned,
           "speedup_vs_loop": loop_ms["median"] / graph_ms["median"],
           "build_plus_generation_ms": build_batched_ms["median"] + best,
           "pairs_per_s": pairs / (best * 1e-3), "images_per_s": total_img / (best * 1e-3),
           "identical": same,
           "tuned": {"group": tuned.group, "num_workgroups": tuned.num_workgroups,
                     "fac_divisor": tuned.fac_divisor, "min_chunk": tuned.min_chunk,
                     "order": tuned.order}}
    for it in items:
        it[0].free()
    return out


# dense fp16 matrix-core peak of the MI355X (no sparsity)
PEAK_MFMA_FP16 = 2.5e15


def adjacent_workloads(torch, si, sg, scene, d_xyz, stream):
    """Mesh resolution (every point of the main scene), normal estimation
    (every point, radius 3x the resolution) and spin-image matching (all
    65,536 images of the 100k-point scene against each other, best match
    per image, then against a fifth of them with every R stored)."""
    out = {}

    def ev_time(fn, reps=5):
        ts = []
        for r in range(1 + reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
        return spread(ts)

    res = si.si_mesh_resolution(scene)
    out["mesh_resolution"] = {"workload": "clustered2m, nearest other point of all 2,000,000",
                              "mean_nn_distance": res,
                              "ms": ev_time(lambda: si.si_mesh_resolution(scene), reps=3)}
    r_n = 3.0 * res
    out["normals"] = {"workload": f"clustered2m, all 2,000,000 points, radius {r_n:.5f} "
                                  "(3x the mesh resolution)",
                      "ms": ev_time(lambda: si.si_estimate_normals(d_xyz, r_n, (20.0, 20.0, 20.0)),
                                    reps=3)}
    cfg = sg.CONFIGS["prims100k"]
    xyz2, nrm2 = sg.config_scene("prims100k")
    p2 = si.Params(cfg.W, cfg.bin, cfg.support_angle)
    sc2 = si.si_build_scene(torch.from_numpy(xyz2).cuda(), torch.from_numpy(nrm2).cuda(),
                            si.si_support_radius(p2))
    idx2 = torch.arange(cfg.N, dtype=torch.int32, device="cuda")
    A, _, _ = si.si_generate(sc2, idx2, p2, si.Sched("fac"))
    n, bins = int(A.shape[0]), cfg.W * cfg.W
    ms_best = ev_time(lambda: si.si_correlate(A, A, R=False))
    _, bi, br = si.si_correlate(A, A, R=False)
    q = A[: n // 5]
    ms_full = ev_time(lambda: si.si_correlate(q, A, R=True, best=False), reps=3)
    flops = 2.0 * n * n * bins
    ach = flops / (ms_best["median"] * 1e-3)
    out["correlation"] = {
        "workload": f"prims100k: {n} spin images (W={cfg.W}) against each other, best match "
                    f"per image; fp16 operands, fp32 sums, on the matrix cores",
        "ms": ms_best, "full_R_ms": ms_full,
        "full_R_workload": f"{n // 5} x {n} pairs, every R stored ({4 * (n // 5) * n / 1e9:.1f} GB)",
        "self_matched": float((bi.cpu() == torch.arange(n)).float().mean()),
        "roofline": {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_MFMA_FP16 / 1e12,
                     "unit": "TFLOP/s", "frac": ach / PEAK_MFMA_FP16,
                     "flops_per_call": flops,
                     "note": "whole call (fp16 conversion of both sets, then the GEMM with "
                             "its epilogue); algorithmic flops 2 n_a n_b N"}}
    del A, q
    sc2.free()
    return out


# The paper's throughput, derived from its weak-scaling text (Section 5.1):
# 64K images in 20.5 s with SS on 160 Xeon E5-2640 cores, every image testing
# all of ~826K points -- end-to-end wall time including MPI.  Context only.
PAPER_TESTS_PER_S_160_CORES_SS = 64_000 * 826_000 / 20.5


def cpu_schedules(oracle, sg, threads, n_images):
    """The paper's experiment on the host cores, as context: the oracle loop
    over the first n_images images of the paper-shaped workload (826K points,
    W = 5, B = 0.1 x mean nearest-neighbour spacing, S = 2 pi, brute force)
    under STATIC, SS, GSS and a FAC2 chunk table, one thread per core."""
    from oracle import chunks as och
    pcfg = sg.CONFIGS["paper826k"]
    xyz, nrm = sg.config_scene("paper826k")
    M = xyz.shape[0]
    B = 0.1 * sg.mean_nn_spacing(xyz)
    n = min(pcfg.N, n_images)
    idx = np.arange(n, dtype=np.int32)
    out = {"workload": f"paper826k loop, its first {n} images (brute force over {M} points, "
                       f"W={pcfg.W}, S=2 pi, FP64 oracle); best of two interleaved rounds",
           "threads": threads}
    # a warm-up call touches every point on every thread
    oracle.generate(xyz, nrm, idx[:threads], pcfg.W, B, pcfg.support_angle, want_touch=False,
                    schedule="static", nthreads=threads)
    best = {}
    for _ in range(2):
        for name in ("static", "ss", "gss", "fac"):
            sch = och.starts(och.fac_sizes(n, threads)) if name == "fac" else name
            t = time.perf_counter()
            oracle.generate(xyz, nrm, idx, pcfg.W, B, pcfg.support_angle, want_touch=False,
                            schedule=sch, nthreads=threads)
            best[name] = min(best.get(name, float("inf")), time.perf_counter() - t)
    for name in ("static", "ss", "gss", "fac"):
        out[name] = {"s": best[name], "pair_tests_per_s": n * M / best[name],
                     "speedup_vs_static": best["static"] / best[name]}
    return out


def paper_shape(torch, si, sg):
    """The shape of the paper's experiments: 826K points, the first 10 %
    oriented, W = 5, B = 0.1 x mean nearest-neighbour spacing, S = 2 pi,
    brute force over all points (a single-cell scene); STATIC, SS and FAC."""
    cfg = sg.CONFIGS["paper826k"]
    xyz, nrm = sg.config_scene("paper826k")
    M, N = xyz.shape[0], cfg.N
    B = 0.1 * sg.mean_nn_spacing(xyz)
    params = si.Params(cfg.W, B, cfg.support_angle)
    scene = si.si_build_scene(torch.from_numpy(xyz).cuda(), torch.from_numpy(nrm).cuda(), 0.0)
    idx = torch.arange(N, dtype=torch.int32, device="cuda")
    img = torch.empty((N, cfg.W, cfg.W), dtype=torch.float32, device="cuda")
    cnt = torch.empty((N,), dtype=torch.int32, device="cuda")
    out = {"workload": f"paper826k: {M} points, first {N} oriented, W={cfg.W}, B={B:.6f} "
                       f"(0.1 x mean nearest-neighbour spacing), S=2 pi, brute force",
           "pair_tests": N * M}
    for kind in ("static", "ss", "fac"):
        sch = si.Sched(kind)
        ms = timed(torch, lambda: si.si_generate(scene, idx, params, sch, img, cnt), reps=5, warm=1)
        out[kind] = {"ms": ms, "pair_tests_per_s": N * M / (ms["median"] * 1e-3),
                     "images_per_s": N / (ms["median"] * 1e-3)}
    out["in_support_pairs"] = int(cnt.to(torch.int64).sum())
    # the same candidate loop with no culling, no angle test and almost no
    # binning: its 13 lane-ops per pair test (3 subtractions, 3 for beta, 3
    # for |d|^2, 1 for alpha^2, 3 comparisons) against the VALU peak
    out["fac"]["test_valu_frac"] = out["fac"]["pair_tests_per_s"] * 13 / PEAK_VALU_OPS
    out["paper_context"] = {
        "pair_tests_per_s": PAPER_TESTS_PER_S_160_CORES_SS,
        "hardware": "160 Xeon E5-2640 cores (8 nodes), MPI, EPSIA-SS, Ramesses ~826K points",
        "ratio_fac_to_paper": out["fac"]["pair_tests_per_s"] / PAPER_TESTS_PER_S_160_CORES_SS}
    scene.free()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the per-image loop would shard over GPUs by ranges of images, each GPU "
              "holding a copy of the scene)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_00901_amd as si
    import scenegen as sg

    dev = torch.device("cuda:0")
    cfg = sg.CONFIGS[args.workload]
    log(f"[bench] generating {cfg.name} (M={cfg.M})")
    xyz, nrm = sg.config_scene(cfg.name)
    M = xyz.shape[0]
    N = cfg.N
    params = si.Params(cfg.W, cfg.bin, cfg.support_angle, "bilinear")
    radius = si.si_support_radius(params)
    d_xyz = torch.from_numpy(xyz).to(dev)
    d_nrm = torch.from_numpy(nrm).to(dev)
    idx = torch.arange(N, dtype=torch.int32, device=dev)
    images = torch.empty((N, cfg.W, cfg.W), dtype=torch.float32, device=dev)
    counts = torch.empty((N,), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    fac = si.Sched("fac")
    main_sched = si.Sched(**MAIN_SCHED)

    def new_events():
        # created (and their HIP events made) outside the timed region: the
        # scene build synchronises, so host work after it delays the kernels
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for e in ev:
            e.record(stream)
        return ev

    def step(ev):
        # e0/e1: the whole generation call (cell ordering + spin kernel);
        # e2/e3: recorded by the library around the spin kernel alone
        scene = si.si_build_scene(d_xyz, d_nrm, radius)
        ev[0].record(stream)
        si.si_set_kernel_events(ev[2], ev[3])
        si.si_generate(scene, idx, params, main_sched, images, counts)
        si.si_set_kernel_events(None, None)
        ev[1].record(stream)
        return scene, ev

    log("[bench] warmup")
    for _ in range(args.warmup):
        step(new_events())
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    events = [new_events() for _ in range(args.steps)]
    scenes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ev in events:
        sc, _ = step(ev)
        scenes.append(sc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    gen_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    kernel_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in events]))
    scene = scenes[-1]
    del scenes
    pairs = int(counts.to(torch.int64).sum().item())
    value = pairs / (ms_step * 1e-3)
    images_per_s = N / (ms_step * 1e-3)
    log(f"[bench] step {ms_step:.2f} ms (generation {gen_ms:.2f} ms, spin kernel {kernel_ms:.2f} ms), "
        f"{pairs} in-support pairs")
    if args.copy_calibration > 0:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {4 * n} bytes for counter calibration")
        del src, dst
    if args.no_extent:
        print(json.dumps({"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
                          "generation_ms": gen_ms, "kernel_ms": kernel_ms, "profiling_run": True}),
              flush=True)
        return

    # ---- workload units for the roofline (outside the timed region) ----
    _, _, st = si.si_generate(scene, idx, params, main_sched, images, counts, stats=True)
    ref_img = images.clone()
    ref_cnt = counts.clone()
    open_params = si.Params(cfg.W, cfg.bin, float(np.float32(math.pi)), "bilinear")
    ext_counts = torch.empty_like(counts)
    ext_img = torch.empty_like(images)
    si.si_generate(scene, idx, open_params, fac, ext_img, ext_counts)
    extent_pairs = int(ext_counts.to(torch.int64).sum().item())
    del ext_img
    ops = OPS_PER_EXTENT_PAIR * extent_pairs + OPS_PER_SUPPORT_PAIR * pairs
    achieved = ops / (kernel_ms * 1e-3)
    # measured device ceilings (the published peak bounds them)
    probes = {k: si.si_peak_probe(k) for k in ("valu", "lds_atomic_seq", "lds_atomic_random",
                                                 "hbm_copy")}
    atomics = ATOMICS_PER_SUPPORT_PAIR * pairs
    traffic = measured_traffic()
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_VALU_OPS / 1e12,
        "unit": "TOP/s",
        "frac": achieved / PEAK_VALU_OPS,
        "traffic": traffic,
        "kernel": "k_spin",
        "kernel_ms": kernel_ms,
        "in_extent_pairs": extent_pairs,
        "in_support_pairs": pairs,
        "pairs_tested": int(st["pairs_tested"]),
        "lds_atomics_per_s": atomics / (kernel_ms * 1e-3),
        "measured_peaks": {"valu_lane_ops_per_s": probes["valu"],
                           "lds_atomics_per_s_conflict_free": probes["lds_atomic_seq"],
                           "lds_atomics_per_s_random_1024_bins": probes["lds_atomic_random"],
                           "hbm_bytes_per_s_copy": probes["hbm_copy"]},
        "frac_of_measured_valu": achieved / probes["valu"],
        "frac_of_measured_lds_atomics": (atomics / (kernel_ms * 1e-3)) / probes["lds_atomic_random"],
        # L2<->fabric bytes per second against an HBM copy: above 1 means most
        # of the traffic is served by the MALL, not HBM
        "fabric_rate_vs_hbm_copy": (traffic / (kernel_ms * 1e-3) / probes["hbm_copy"]
                                    if traffic else None),
        # T_roof = max(algorithmic VALU work / measured VALU peak,
        #              LDS atomics / measured random-bin atomic peak)
        "t_roof_ms": 1e3 * max(ops / probes["valu"], atomics / probes["lds_atomic_random"]),
    }
    roofline["frac_of_t_roof"] = roofline["t_roof_ms"] / kernel_ms

    # ---- learned cost model ----
    model, cm_info = None, None
    if not args.no_schedules:
        log("[bench] training the cost model")
        model, cm_info = train_cost_model(
            torch, si, sg, {"scene": scene, "idx": idx, "params": params, "counts": ref_cnt})
        log(f"[bench] cost model: {cm_info['mae_test']:.1f} held-out MAE "
            f"(untrained {cm_info['mae_test_untrained']:.1f})")

    # ---- every schedule, generation only, bit-identical images ----
    sched_res = {}
    if not args.no_schedules:
        # the four techniques of the paper on the spread cell order (default)
        # and on the contiguous cell order; LEARNED builds its own order
        runs = [(k, k, "spread") for k in ("static", "ss", "gss", "fac")]
        runs += [(k + "_cell", k, "cell") for k in ("static", "ss", "gss", "fac")]
        runs += [("learned", "learned", "spread")]
        # small chunks over the cell order: every workgroup sweeps the scene
        # at once (the main step's schedule, and self-scheduling of 32)
        runs += [("fac_sweep", "fac", "cell"), ("ss_sweep", "ss", "cell")]
        # two later techniques of the family: TSS, and probabilistic factoring
        # fed with sigma / mu of the per-image cost (the cost model's predicted
        # in-support counts + 1; the measured counts without a model)
        cost = ref_cnt.to(torch.float64) + 1.0
        cv_source = "measured in-support counts + 1"
        if model is not None:
            pred = si.si_cost_model_predict(model, si.si_features(scene, idx, params))
            cost = pred.to(torch.float64).clamp_min(0.0) + 1.0
            cv_source = "cost model's predicted in-support counts + 1"
        cost_cv = float(cost.std() / cost.mean())
        del cost
        runs += [("tss", "tss", "spread"), ("fac_prob", "fac_prob", "spread")]
        # three whose chunk the claiming workgroup sizes (instrumented build of
        # the kernel: per-group timing): weighted, adaptive weighted, adaptive
        runs += [("wf", "wf", "spread"), ("awf", "awf", "spread"), ("af", "af", "spread")]
        for name, kind, order in runs:
            sch = si.Sched(kind, model=model if kind == "learned" else None, order=order,
                           fac_divisor=cost_cv if kind == "fac_prob" else 0.0)
            if name == "fac_sweep":
                sch = main_sched
            elif name == "ss_sweep":
                sch = si.Sched("ss", min_chunk=32, order="cell")
            times, used, ok = [], None, True
            for r in range(WARM + REPS):
                images.fill_(-1.0)
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                ev[0].record(stream)
                _, _, s2 = si.si_generate(scene, idx, params, sch, images, counts, stats=True)
                ev[1].record(stream)
                torch.cuda.synchronize()
                used = s2["sched_used"]
                ok = ok and bool(torch.equal(images, ref_img) and torch.equal(counts, ref_cnt))
                if r >= WARM:
                    times.append((s2["kernel_ms"], ev[0].elapsed_time(ev[1])))
            busy = s2["wg_busy_ns"].astype(np.float64)
            call = spread([t[1] for t in times])
            sched_res[name] = {"order": order if kind != "learned" else "learned",
                               "kernel_ms": spread([t[0] for t in times]), "call_ms": call,
                               "pairs_per_s": pairs / (call["median"] * 1e-3),
                               "images_per_s": N / (call["median"] * 1e-3),
                               "identical": ok, "sched_used": list(si.SCHED)[used],
                               "n_chunks": s2["n_chunks"],
                               "imbalance": float(busy.max() / max(busy.mean(), 1.0))}
            log(f"[bench] {name}: kernel {sched_res[name]['kernel_ms']['median']:.2f} ms, "
                f"call {call['median']:.2f} ms, identical {ok}, "
                f"imbalance {sched_res[name]['imbalance']:.3f}")
        sched_res["fac_prob"]["cost_cv"] = cost_cv
        sched_res["fac_prob"]["cost_cv_source"] = cv_source
        # the learned schedule against FAC2, same workgroups and group size
        if "learned" in sched_res:
            lk, fk = sched_res["learned"], sched_res["fac"]
            sched_res["learned_vs_fac"] = {
                "kernel_ratio": lk["kernel_ms"]["median"] / fk["kernel_ms"]["median"],
                "call_ratio": lk["call_ms"]["median"] / fk["call_ms"]["median"],
                "plan_ms": lk["call_ms"]["median"] - lk["kernel_ms"]["median"] -
                           (fk["call_ms"]["median"] - fk["kernel_ms"]["median"])}
        base = sched_res["static"]["call_ms"]["median"]
        base_cell = sched_res["static_cell"]["call_ms"]["median"]
        for k in sched_res:
            if "call_ms" not in sched_res[k]:
                continue
            sched_res[k]["speedup_vs_static"] = base / sched_res[k]["call_ms"]["median"]
            if k.endswith("_cell"):
                sched_res[k]["speedup_vs_static_cell"] = base_cell / sched_res[k]["call_ms"]["median"]
        si.si_generate(scene, idx, params, fac, images, counts)

    # ---- heterogeneous workers, emulated (the paper's Section 5.2 setting) ----
    hetero = None
    if not args.no_schedules:
        kinds = ("static", "ss", "gss", "fac", "tss", "fac_prob", "learned", "wf", "awf", "af")
        hetero = {"setting": "every 2nd workgroup 2x slower: after each group of images it "
                             "spends the group's own time again, idling (CU free) or with every "
                             "thread spinning on arithmetic (CU busy); same images",
                  "slowdown": 2.0, "every": 2}

        def hetero_run(kind, reps=5):
            sch = si.Sched(kind, model=model if kind == "learned" else None,
                           fac_divisor=cost_cv if kind == "fac_prob" else 0.0)
            ks, ok = [], True
            for r in range(2 + reps):
                _, _, s2 = si.si_generate(scene, idx, params, sch, images, counts, stats=True)
                ok = ok and bool(torch.equal(counts, ref_cnt))
                if r >= 2:
                    ks.append(s2["kernel_ms"])
            busy = s2["wg_busy_ns"].astype(np.float64)
            return {"kernel_ms": spread(ks), "counts_identical": ok,
                    "imbalance": float(busy.max() / max(busy.mean(), 1.0))}

        try:
            si.si_set_emulated_workers(2, 2.0)
            for model_name, busy_mode in (("idle", False), ("busy", True)):
                si.si_set_emulated_mode(busy_mode, "every")
                res = {k: hetero_run(k) for k in kinds}
                for k in kinds:
                    res[k]["speedup_vs_static"] = (res["static"]["kernel_ms"]["median"] /
                                                   res[k]["kernel_ms"]["median"])
                hetero[model_name] = res
                log(f"[bench] heterogeneous ({model_name}): " + ", ".join(
                    f"{k} {res[k]['kernel_ms']['median']:.2f} ms" for k in kinds))
            # the claim-order effect (Section 5.2): slow workgroups first or
            # last to claim, GSS against FAC2
            order = {}
            for model_name, busy_mode in (("idle", False), ("busy", True)):
                o = {}
                for place in ("first", "last"):
                    si.si_set_emulated_mode(busy_mode, place)
                    for k in ("gss", "fac"):
                        o[f"{k}_{place}"] = hetero_run(k, reps=3)["kernel_ms"]
                for k in ("gss", "fac"):
                    o[f"{k}_first_over_last"] = o[f"{k}_first"]["median"] / o[f"{k}_last"]["median"]
                order[model_name] = o
                log(f"[bench] claim order ({model_name}): GSS first/last "
                    f"{o['gss_first_over_last']:.3f}, FAC {o['fac_first_over_last']:.3f}")
            hetero["claim_order"] = order
        finally:
            si.si_set_emulated_workers(0, 1.0)
            si.si_set_emulated_mode(False, "every")
    torch.cuda.synchronize()
    del ref_img, ref_cnt

    # ---- next to the path: mesh resolution, normals, spin-image matching ----
    adjacent = None
    if not args.no_adjacent:
        adjacent = adjacent_workloads(torch, si, sg, scene, d_xyz, stream)
        log(f"[bench] adjacent: {adjacent}")

    # ---- batching ----
    batch = None
    if not args.no_batch:
        log("[bench] batched: 256 scenes")
        batch = batched(torch, si, sg, model)
        log(f"[bench] batched: {batch}")

    # ---- the paper's workload shape (context) ----
    paper = None
    if not args.no_paper_shape:
        log("[bench] paper-shape run")
        paper = paper_shape(torch, si, sg)
        log(f"[bench] paper shape: FAC {paper['fac']['pair_tests_per_s']:.3g} pair tests/s "
            f"({paper['paper_context']['ratio_fac_to_paper']:.0f}x the paper's 160 cores)")

    # ---- FP64 CPU oracle on a bounded sample of the main workload ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        threads = oracle.max_threads()
        order = np.random.default_rng(12345).permutation(N)

        def sample_rate(seconds, grid):
            # batches of seeded-random images until `seconds` of CPU work
            done, dt, pairs_cpu = 0, 0.0, 0
            batch_n = threads * (64 if grid else 4)
            while dt < seconds and done < N:
                sample = order[done:done + batch_n]
                t = time.perf_counter()
                r = oracle.generate(xyz, nrm, sample, cfg.W, cfg.bin, cfg.support_angle,
                                    want_touch=False, grid=grid)
                el = time.perf_counter() - t
                dt += el
                done += len(sample)
                pairs_cpu += int(r["cnt_sure"].sum() + r["cnt_amb"].sum())
                left = seconds - dt
                batch_n = int(min(max(threads, len(sample) * max(left, 0.5) / max(el, 1e-3)),
                                  400000))
            return done, dt, pairs_cpu

        # the oracle's cell-grid form: the same pairs as brute force over the
        # 7 x 7 x 7 cells around each image's point, the algorithm the GPU runs
        done, dt, pairs_cpu = sample_rate(args.cpu_seconds, True)
        log(f"[bench] cpu oracle (grid): {done} images, {threads} threads, {dt:.1f} s")
        cpu = {"value": float(pairs_cpu / dt), "unit": "pairs/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "sample": f"{done} seeded-random images of {cfg.name}, FP64 oracle in its cell-grid "
                         f"form (the pairs of the 7 x 7 x 7 cells around each image's point, grid "
                         f"built in each call), {dt:.1f} s",
               "images_per_s": done / dt}
        # and its brute-force form (every image against all M points)
        done, dt, pairs_cpu = sample_rate(max(3.0, args.cpu_seconds / 3), False)
        log(f"[bench] cpu oracle (brute force): {done} images, {dt:.1f} s")
        cpu["brute_force"] = {"pairs_per_s": float(pairs_cpu / dt), "images_per_s": done / dt,
                              "sample": f"{done} seeded-random images, brute force over all "
                                        f"{M} points each, FP64, {dt:.1f} s"}
        # one thread on the 2,000-point sphere workload (all 2,000 images, brute force)
        c1 = sg.CONFIGS["sphere2k"]
        sxyz, snrm = sg.config_scene("sphere2k")
        t = time.perf_counter()
        r1 = oracle.generate(sxyz, snrm, np.arange(c1.N, dtype=np.int32), c1.W, c1.bin,
                             c1.support_angle, want_touch=False, nthreads=1)
        el = time.perf_counter() - t
        cpu["single_thread_sphere2k"] = {
            "pairs_per_s": float((r1["cnt_sure"].sum() + r1["cnt_amb"].sum()) / el),
            "pair_tests_per_s": c1.N * sxyz.shape[0] / el, "s": el, "threads": 1}
        if args.cpu_sched_images > 0:
            cpu["schedules"] = cpu_schedules(oracle, sg, threads, args.cpu_sched_images)
            log("[bench] cpu schedules: " + ", ".join(
                f"{k} {v['s']:.2f} s" for k, v in cpu["schedules"].items()
                if isinstance(v, dict)))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {M} points, {N} oriented, W={cfg.W}, bin={cfg.bin}, "
                               f"support angle 60 deg, bilinear, cell list, "
                               f"{MAIN_SCHED_DESC}",
                   "global_batch": N, "parallelism": "single GPU, persistent workgroups"},
        "images_per_s": images_per_s,
        "generation_ms": gen_ms,
        "schedules": sched_res,
        "heterogeneous_emulated": hetero,
        "cost_model": cm_info,
        "adjacent": adjacent,
        "batched": batch,
        "paper_shape": paper,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
