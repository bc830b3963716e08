"""Throughput of the moving image-source synthesis on one MI355X.

A step is one forward synthesis of the whole workload (delay tracks, gather-
reduce over images x outputs x taps, group reduction) with the source signal
already resident in HBM.  Prints one JSON line.

Metric: image-sample taps/s = sum over scenes, mics, images of (n_in + T - 1) * T
taps per step / seconds per step.  Forward+backward counts four tap chains
per forward tap (forward, dL/dx, the h chain and the h' chain of the gain and
delay adjoints).
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
FLOPS_PER_TAP = 4         # two FMAs per tap (the two interpolation rows of the table, each multiply-added)

WORKLOADS = {
    "config2": ("paper-scale plain: 8x6x3.5 m room, K=12 (2625 images), 4 s at 16 kHz, "
                "tiers 16k/1k/100 Hz, T=64, 1 mic", G.config2),
    "config1": ("tiny plain: 5x4x3 m room, K=2 (25 images), 1 s at 16 kHz, full rate, T=32, 1 mic", G.config1),
}


def cpu_baseline(scenes, par, target_s: float = 15.0):
    """The FP64 oracle on the host cores, on a bounded sample of output samples
    of the first scene (tier-emulating mode, every image, exact kernel)."""
    from oracle import oracle as O
    sc = scenes[0]
    rng = np.random.default_rng(123)
    n_img = O.count_images(sc.max_order)
    n = 64
    t0 = time.perf_counter()
    O.forward(sc, par, idx=np.sort(rng.choice(sc.n_out, n, replace=False)))
    dt = time.perf_counter() - t0
    n = int(max(64, min(sc.n_out, n * target_s / max(dt, 1e-3))))
    idx = np.sort(rng.choice(sc.n_out, n, replace=False))
    t0 = time.perf_counter()
    O.forward(sc, par, idx=idx)
    dt = time.perf_counter() - t0
    taps = float(n) * sc.n_mics * n_img * par.taps
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": taps / dt, "unit": "taps/s", "cores": cores, "kind": "oracle",
            "sample": "%d random output samples x %d images x %d taps of the first scene "
                      "(FP64, exact kernel, tier-emulating delays), %.1f s" % (n, n_img, par.taps, dt)}


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the fwd+bwd and batched measurements")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB: the reference kernel that "
                         "scales the HBM byte counters of a profiler run")
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

    # per-kernel durations from HIP events on the launch stream
    plan.profile_begin()
    sec_prof = timed(lambda: plan.forward(x, y), args.steps, torch)
    prof = plan.profile_end()
    sec = min(sec_prof, timed(lambda: plan.forward(x, y), args.steps, torch))
    ms = sec * 1e3
    taps = plan.forward_taps
    synth_ms = prof["synth_ms"] / max(1, prof["synth_launches"])
    launches_per_step = prof["synth_launches"] / args.steps
    achieved = taps / launches_per_step * FLOPS_PER_TAP / (synth_ms * 1e-3)
    rec = {
        "metric": "image-sample taps/s (forward synthesis, plain path)",
        "value": taps / sec,
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

    if not args.no_extra:
        # forward + backward (dL/dx, dL/dbeta, dL/dknots) on the same workload
        gy = torch.randn(plan.y_total, generator=torch.Generator().manual_seed(1)).cuda()

        def fwd_bwd():
            plan.forward(x, y)
            plan.backward(x, gy)
        fwd_bwd()
        plan.profile_begin()
        sec_fb = timed(fwd_bwd, max(3, args.steps // 4), torch)
        pb = plan.profile_end()
        nfb = max(3, args.steps // 4)
        rec["fwd_bwd"] = {"value": 4 * taps / sec_fb, "unit": "taps/s", "ms_per_step": sec_fb * 1e3,
                          "phases_ms_per_step": {k[:-3]: pb[k] / nfb for k in
                                                 ("tracks_ms", "synth_ms", "reduce_ms", "adjoint_ms", "params_ms")}}
        del plan, x, y, gy
        torch.cuda.empty_cache()

        # batched vs plain on the 256-scene workload
        s3, p3 = G.config3()
        plan3 = Plan(s3, p3)
        x3 = plan3.pack_x([s.x for s in s3])
        tune = plan3.autotune(x3)
        torch.cuda.empty_cache()
        y3 = torch.empty(plan3.y_total, dtype=torch.float32, device="cuda")
        plan3.forward_batched(x3, y3)
        nb = max(3, args.steps // 4)
        sec_b = timed(lambda: plan3.forward_batched(x3, y3), nb, torch)
        plan3.profile_begin()
        timed(lambda: plan3.forward_batched(x3, y3, graph=False), 2, torch)
        pb3 = plan3.profile_end()
        plan3.forward(x3, y3)
        sec_p = timed(lambda: plan3.forward(x3, y3), 2, torch)
        t3 = plan3.forward_taps
        rec["batched"] = {"workload": "config3: 256 scenes, rooms U(3,10)xU(3,8)xU(2.5,4) m, Sabine orders 6-18, "
                                      "1-8 s at 16 kHz, lines and circles, tiers, T=64",
                          "images": int(plan3.n_images.sum()), "taps_per_step": t3,
                          "value": t3 / sec_b, "unit": "taps/s", "ms_per_step": sec_b * 1e3,
                          "plain_value": t3 / sec_p, "plain_ms_per_step": sec_p * 1e3,
                          "speedup_vs_plain": sec_p / sec_b,
                          "persistent_kernel_ms": pb3["synth_ms"] / max(1, pb3["synth_launches"]),
                          "persistent_frac_of_fp32_peak": t3 * FLOPS_PER_TAP /
                          (pb3["synth_ms"] / max(1, pb3["synth_launches"]) * 1e-3) / PEAK_FP32,
                          "tuning": tune}
        del plan3, x3, y3
        torch.cuda.empty_cache()

    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(scenes, par)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
