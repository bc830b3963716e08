"""Throughput of the moving image-source synthesis on one MI355X.

A step is one forward synthesis of the whole workload (delay tracks, gather-
reduce over images x outputs x taps, group reduction) with the source signal
already resident in HBM.  Prints one JSON line.

Metric: image-sample taps/s = sum over scenes, mics, images of (n_in + T - 1) * T
taps per step / seconds per step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2508_03065_amd import scenegen as G  # noqa: E402

PEAK_FP32 = 157.3e12      # MI355X FP32 vector, FLOP/s
FLOPS_PER_TAP = 4         # two FMAs per tap (table interpolation and multiply-accumulate)

WORKLOADS = {
    "config2": ("paper-scale plain: 8x6x3.5 m room, K=12 (2625 images), 4 s at 16 kHz, "
                "tiers 16k/1k/100 Hz, T=64, 1 mic", G.config2),
    "config1": ("tiny plain: 5x4x3 m room, K=2 (25 images), 1 s at 16 kHz, full rate, T=32, 1 mic", G.config1),
}


def cpu_baseline(scenes, par, target_s: float = 12.0):
    """The FP64 oracle on the host cores, on a bounded sample of output samples
    of the first scene (tier-emulating mode, every image, exact kernel)."""
    from oracle import oracle as O
    sc = scenes[0]
    rng = np.random.default_rng(123)
    n_img = O.count_images(sc.max_order)
    n = 8
    t0 = time.perf_counter()
    O.forward(sc, par, idx=np.sort(rng.choice(sc.n_out, n, replace=False)))
    dt = time.perf_counter() - t0
    n = int(max(8, min(sc.n_out, n * target_s / max(dt, 1e-3))))
    idx = np.sort(rng.choice(sc.n_out, n, replace=False))
    t0 = time.perf_counter()
    O.forward(sc, par, idx=idx)
    dt = time.perf_counter() - t0
    taps = float(n) * sc.n_mics * n_img * par.taps
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": taps / dt, "unit": "taps/s", "cores": cores, "kind": "oracle",
            "sample": "%d random output samples x %d images x %d taps of the first scene "
                      "(FP64, exact kernel, tier-emulating delays), %.1f s" % (n, n_img, par.taps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(scenes or output tiles would shard with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_03065_amd.msim import Plan

    desc, gen = WORKLOADS[args.workload]
    scenes, par = gen()
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        plan.forward(x, y)
    torch.cuda.synchronize()
    if plan.device_status() != 0:
        raise RuntimeError("device status flags set")

    plan.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(x, y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_end()
    # timing run without per-launch events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(x, y)
    torch.cuda.synchronize()
    wall = min(wall, time.perf_counter() - t0)

    ms = wall * 1e3 / args.steps
    taps = plan.forward_taps
    synth_ms = prof["synth_ms"] / max(1, prof["synth_launches"])
    launches_per_step = prof["synth_launches"] / args.steps
    achieved = taps / launches_per_step * FLOPS_PER_TAP / (synth_ms * 1e-3)
    rec = {
        "metric": "image-sample taps/s (forward synthesis, plain path)",
        "value": taps / (ms * 1e-3),
        "unit": "taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded N(0,1) source, seeded trajectories and walls)",
        "config": {"workload": args.workload + ": " + desc, "scenes": len(scenes),
                   "images": int(plan.n_images.sum()), "taps_per_step": taps},
        "phases_ms_per_step": {k[:-3]: prof[k] / args.steps for k in ("tracks_ms", "synth_ms", "reduce_ms")},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": None,
                     "kernel": "k_synth_fwd", "kernel_ms": synth_ms},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(scenes, par)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
