"""Spin-image generation benchmark on one MI355X.

Workload (seeded, synthetic): the clustered primitives scene -- 2,000,000
float32 oriented points on 400 random tori and ellipsoids whose centres are
Gaussian-clustered (sigma 1) in a [0, 40]^3 box, per-object density varying
tenfold -- with every point oriented, W = 32, bin 0.02, support angle 60
degrees, bilinear binning, FAC chunking on the persistent kernel.

One step = the whole hot path: si_build_scene (bounding box, cell binning,
scan, scatter) followed by si_generate (FAC chunk claims, candidate culling,
pair tests, LDS accumulation, image write-back), inputs already resident in
HBM.  Reported value: in-support point pairs binned per second; also images
per second, the generation-only time of every schedule with its speedup over
STATIC (images bit-identical), the roofline of the spin kernel and the FP64
CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
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

# Algorithmic work per unit (VALU lane operations and LDS atomics), counted on
# the definition rather than on executed instructions:
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
# flops and needs packed dual FP32, which this build does not emit).
PEAK_VALU_OPS = 256 * 64 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="clustered2m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-schedules", action="store_true")
    ap.add_argument("--no-extent", action="store_true",
                    help="skip the extra launches that count in-extent pairs (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the per-image loop would shard over GPUs as described in DESIGN.md)",
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

    def step():
        # e0/e1: the whole generation call (cell ordering + spin kernel);
        # k0/k1: recorded by the library around the spin kernel alone
        scene = si.si_build_scene(d_xyz, d_nrm, radius)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        si.si_set_kernel_events(ev[2], ev[3])
        si.si_generate(scene, idx, params, fac, images, counts)
        si.si_set_kernel_events(None, None)
        ev[1].record(stream)
        return scene, ev

    log("[bench] warmup")
    for _ in range(args.warmup):
        sc, _ = step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    events = []
    scenes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sc, ev = step()
        events.append(ev)
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

    if args.no_extent:
        print(json.dumps({"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
                          "generation_ms": gen_ms, "kernel_ms": kernel_ms, "profiling_run": True}),
              flush=True)
        return
    # ---- workload units for the roofline (outside the timed region) ----
    _, _, st = si.si_generate(scene, idx, params, fac, images, counts, stats=True)
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
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_VALU_OPS / 1e12,
        "unit": "TOP/s",
        "frac": achieved / PEAK_VALU_OPS,
        "traffic": None,
        "kernel": "k_spin",
        "kernel_ms": kernel_ms,
        "in_extent_pairs": extent_pairs,
        "in_support_pairs": pairs,
        "pairs_tested": int(st["pairs_tested"]),
        "lds_atomics_per_s": ATOMICS_PER_SUPPORT_PAIR * pairs / (kernel_ms * 1e-3),
    }

    # ---- every schedule, generation only, bit-identical images ----
    sched_res = {}
    if not args.no_schedules:
        for kind in ["static", "ss", "gss", "fac", "learned"]:
            sch = si.Sched(kind)
            times = []
            ok = True
            used = None
            for r in range(4):
                _, _, s2 = si.si_generate(scene, idx, params, sch, images, counts, stats=True)
                used = s2["sched_used"]
                if r:
                    times.append(s2["kernel_ms"])
            busy = s2["wg_busy_ns"].astype(np.float64)
            ok = bool(torch.equal(images, ref_img) and torch.equal(counts, ref_cnt))
            sched_res[kind] = {"ms": float(np.median(times)), "identical": ok,
                               "sched_used": list(si.SCHED)[used], "n_chunks": s2["n_chunks"],
                               "imbalance": float(busy.max() / max(busy.mean(), 1.0))}
            log(f"[bench] {kind}: {sched_res[kind]}")
        base = sched_res["static"]["ms"]
        for k in sched_res:
            sched_res[k]["speedup_vs_static"] = base / sched_res[k]["ms"]
        si.si_generate(scene, idx, params, fac, images, counts)
    torch.cuda.synchronize()

    # ---- FP64 CPU oracle on a bounded sample of the same workload ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        threads = oracle.max_threads()
        rng = np.random.default_rng(12345)
        probe = rng.choice(N, size=threads * 2, replace=False)
        t = time.perf_counter()
        r = oracle.generate(xyz, nrm, probe, cfg.W, cfg.bin, cfg.support_angle, want_touch=False)
        per_img = (time.perf_counter() - t) / len(probe)
        n_s = int(max(threads, min(N, args.cpu_seconds / max(per_img, 1e-6))))
        sample = rng.choice(N, size=n_s, replace=False)
        log(f"[bench] cpu oracle on {n_s} images, {threads} threads")
        t = time.perf_counter()
        r = oracle.generate(xyz, nrm, sample, cfg.W, cfg.bin, cfg.support_angle, want_touch=False)
        dt = time.perf_counter() - t
        cpu = {"value": float(r["cnt_sure"].sum() / dt), "unit": "pairs/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{n_s} seeded-random images of {cfg.name} (brute force over all {M} "
                         f"points each, FP64), {dt:.1f} s",
               "images_per_s": n_s / dt}

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
                               f"support angle 60 deg, bilinear, FAC, cell list",
                   "global_batch": N, "parallelism": "single GPU, persistent workgroups"},
        "images_per_s": images_per_s,
        "generation_ms": gen_ms,
        "schedules": sched_res,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
