"""Throughput of the moving image-source synthesis on one MI355X.

A step is one forward synthesis of the whole workload (delay tracks, gather-
reduce over images x outputs x taps, group reduction) with the source signal
already resident in HBM.  Prints one JSON line.

Metric: image-sample taps/s = sum over scenes, mics, images of (n_in + T - 1) * T
taps per step / seconds per step.  Forward+backward counts four tap chains
per forward tap (forward, dL/dx, the h chain and the h' chain of the gain and
delay adjoints).  The Farrow form computes the same output (within the same
tolerance) without visiting every tap; its rate is quoted in the same
equivalent taps/s, and its kernel roofline uses the work it really does.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2508_03065_amd import scenegen as G  # noqa: E402

PEAK_FP32 = 157.3e12      # MI355X FP32 vector, FLOP/s
PEAK_LDS = 256 * 256 * 2.4e9   # LDS reads, B/s: 256 CUs x 256 B/clk (b128) x 2.4 GHz
FLOPS_PER_TAP = 4         # table form: two FMAs per tap (the interpolated coefficient, the multiply-add)


def table_lds_per_tap(outputs_per_lane: int) -> float:
    """Table form, LDS bytes per tap: the source sample and the row's two FP32 and one
    FP16 quadratic-table values (14 B); with two adjacent outputs per lane one table
    read and one new source quad serve both outputs' taps (7 B)."""
    return 14.0 / outputs_per_lane


def farrow_lds_per_sample(order: int) -> int:
    """Farrow form: the M+1 filtered values read per image sample (40 B for M <= 9)."""
    return 40 if order <= 9 else 48


def farrow_flops_per_sample(order: int) -> int:
    """Farrow form, per image sample: Horner of degree M (M FMAs), the cubic delay
    offset (3 FMAs), and the gain times the polynomial added to the output (1 FMA)."""
    return 2 * (order + 3 + 1)


WORKLOADS = {
    "config2": ("paper-scale plain: 8x6x3.5 m room, K=12 (2625 images), 4 s at 16 kHz, "
                "tiers 16k/1k/100 Hz, T=64, 1 mic", G.config2),
    "config1": ("tiny plain: 5x4x3 m room, K=2 (25 images), 1 s at 16 kHz, full rate, T=32, 1 mic", G.config1),
}
FD_KINDS = {"table": 0, "farrow": 1}
KERNEL_OF = {"table": ("k_synth_fwd", "msim_kernels.hip"), "farrow": ("k_farrow_fwd", "msim_farrow.hip")}


def with_fd(par, fd: str):
    import dataclasses
    return dataclasses.replace(par, fd_kind=FD_KINDS[fd])


def source_sha(fname: str) -> str:
    with open(os.path.join(ROOT, "paper_2508_03065_amd", "csrc", fname), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def pmc_traffic(kernel: str, workload: str, src: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>__<workload>__hbm_pmc.md (FETCH_SIZE and WRITE_SIZE, scaled by
    the copy-kernel factors recorded there), or None when there is none or the
    kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s__%s__hbm_pmc.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    tb = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not sha or not tb or sha.group(1) != source_sha(src):
        return None
    return float(tb.group(1))


def cpu_baseline(scenes, par, target_s: float = 15.0):
    """The FP64 oracle on the host cores, on a bounded sample of output samples
    of the first scene (tier-emulating mode, every image, exact kernel)."""
    from oracle import oracle as O
    sc = scenes[0]
    rng = np.random.default_rng(123)
    n_img = O.count_images(sc.max_order)
    n, dt = 256, 0.0
    while True:
        idx = np.sort(rng.choice(sc.n_out, n, replace=False))
        t0 = time.perf_counter()
        O.forward(sc, par, idx=idx)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * target_s or n >= sc.n_out:
            break
        n = int(min(sc.n_out, max(2 * n, n * target_s / max(dt, 1e-3))))
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


def measure_forward(plan, x, y, steps, torch):
    """Seconds per plain forward step, and the per-kernel HIP-event profile."""
    plan.profile_begin()
    sec_prof = timed(lambda: plan.forward(x, y), steps, torch)
    prof = plan.profile_end()
    sec = min(sec_prof, timed(lambda: plan.forward(x, y), steps, torch))
    return sec, prof


def synth_roofline(plan, prof, steps, fd, par, workload):
    kernel, src = KERNEL_OF[fd]
    taps = plan.forward_taps
    kms = prof["synth_ms"] / max(1, prof["synth_launches"])
    per_step = prof["synth_launches"] / steps
    if fd == "table":
        flops = taps / per_step * FLOPS_PER_TAP
        lds = taps / per_step * table_lds_per_tap(plan.tuning()["outputs_per_lane"])
    else:
        flops = taps / par.taps / per_step * farrow_flops_per_sample(par.farrow_order)
        lds = taps / par.taps / per_step * farrow_lds_per_sample(par.farrow_order)
    achieved = flops / (kms * 1e-3)
    traffic = pmc_traffic(kernel, workload, src)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "traffic": traffic, "kernel": kernel, "kernel_ms": kms,
            "flops_per_launch": flops,
            "lds": {"achieved": lds / (kms * 1e-3) / 1e12, "peak": PEAK_LDS / 1e12, "unit": "TB/s",
                    "frac": lds / (kms * 1e-3) / PEAK_LDS, "bytes_per_launch": lds}}


def measure_fwd_bwd(plan, x, y, steps, torch):
    gy = torch.randn(plan.y_total, generator=torch.Generator().manual_seed(1)).cuda()

    def fwd_bwd():
        plan.forward(x, y)
        plan.backward(x, gy)
    fwd_bwd()
    plan.profile_begin()
    sec = timed(fwd_bwd, steps, torch)
    pb = plan.profile_end()
    return {"value": 4 * plan.forward_taps / sec, "unit": "taps/s", "ms_per_step": sec * 1e3,
            "phases_ms_per_step": {k[:-3]: pb[k] / steps for k in
                                   ("tracks_ms", "synth_ms", "reduce_ms", "adjoint_ms", "params_ms", "filter_ms")}}


def measure_batched(scenes, par, steps, torch):
    from paper_2508_03065_amd.msim import Plan
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    tune = plan.autotune(x)
    torch.cuda.empty_cache()
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
    plan.forward_batched(x, y)
    sec_b = timed(lambda: plan.forward_batched(x, y), steps, torch)
    plan.profile_begin()
    timed(lambda: plan.forward_batched(x, y, graph=False), 2, torch)
    pb = plan.profile_end()
    plan.forward(x, y)
    sec_p = timed(lambda: plan.forward(x, y), 2, torch)
    t = plan.forward_taps
    out = {"images": int(plan.n_images.sum()), "taps_per_step": t,
           "value": t / sec_b, "unit": "taps/s", "ms_per_step": sec_b * 1e3,
           "plain_value": t / sec_p, "plain_ms_per_step": sec_p * 1e3, "speedup_vs_plain": sec_p / sec_b,
           "persistent_kernel_ms": pb["synth_ms"] / max(1, pb["synth_launches"]), "tuning": tune}
    del plan, x, y
    torch.cuda.empty_cache()
    return out


def measure_differentiation(fd, steps, torch):
    """Forward (batched, graph-replayed) + backward of the 32-scene differentiation
    workload with L = 0.5 ||y - target||^2: gradients for x, the 6 wall
    coefficients of every scene and the 8 source knots of every scene."""
    from paper_2508_03065_amd.msim import Plan
    scenes, par = G.config4()
    plan = Plan(scenes, with_fd(par, fd))
    x = plan.pack_x([s.x for s in scenes])
    g = torch.Generator().manual_seed(4)
    target = (0.01 * torch.randn(plan.y_total, generator=g)).cuda()
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")

    def step():
        plan.forward_batched(x, y)
        plan.backward(x, y - target)
    step()
    plan.profile_begin()
    sec = timed(step, steps, torch)
    pb = plan.profile_end()
    out = {"value": 4 * plan.forward_taps / sec, "unit": "taps/s", "ms_per_step": sec * 1e3,
           "scenes": len(scenes), "images": int(plan.n_images.sum()), "taps_per_step": 4 * plan.forward_taps,
           "phases_ms_per_step": {k[:-3]: pb[k] / steps for k in
                                  ("graph_ms", "tracks_ms", "adjoint_ms", "params_ms", "reduce_ms", "filter_ms")}}
    del plan, x, y, target
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed forward steps first (the GPU clocks take a few hundred ms to settle)")
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--fd", default="table", choices=sorted(FD_KINDS),
                    help="fractional-delay form of the headline measurement (the other is reported beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other form, fwd+bwd and batched measurements")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB: the reference kernel that "
                         "scales the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(scenes or output tiles would shard with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_03065_amd.msim import Plan

    desc, gen = WORKLOADS[args.workload]
    scenes, par0 = gen()
    par = with_fd(par0, args.fd)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        plan.forward(x, y)
    torch.cuda.synchronize()
    if plan.device_status() != 0:
        raise RuntimeError("device status flags set")

    sec, prof = measure_forward(plan, x, y, args.steps, torch)
    taps = plan.forward_taps
    rec = {
        "metric": "image-sample taps/s (forward synthesis, plain path, %s form of the fractional delay)" % args.fd,
        "value": taps / sec,
        "unit": "taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded N(0,1) source, seeded trajectories and walls)",
        "config": {"workload": args.workload + ": " + desc, "fd": args.fd, "scenes": len(scenes),
                   "images": int(plan.n_images.sum()), "taps_per_step": taps},
        "phases_ms_per_step": {k[:-3]: prof[k] / args.steps
                               for k in ("tracks_ms", "synth_ms", "reduce_ms", "filter_ms")},
        "roofline": synth_roofline(plan, prof, args.steps, args.fd, par, args.workload),
    }

    if not args.no_extra:
        nfb = max(3, args.steps // 4)
        rec["fwd_bwd"] = measure_fwd_bwd(plan, x, y, nfb, torch)
        del plan
        torch.cuda.empty_cache()
        # the other fractional-delay form on the same workload
        other = "farrow" if args.fd == "table" else "table"
        po = with_fd(par0, other)
        plan = Plan(scenes, po)
        for _ in range(args.warmup):
            plan.forward(x, y)
        so, pro = measure_forward(plan, x, y, args.steps, torch)
        rec[other] = {"value": taps / so, "unit": "taps/s", "ms_per_step": so * 1e3,
                      "phases_ms_per_step": {k[:-3]: pro[k] / args.steps
                                             for k in ("tracks_ms", "synth_ms", "reduce_ms", "filter_ms")},
                      "roofline": synth_roofline(plan, pro, args.steps, other, po, args.workload),
                      "fwd_bwd": measure_fwd_bwd(plan, x, y, nfb, torch)}
        del plan, x, y
        torch.cuda.empty_cache()

        # batched vs plain on the 256-scene workload, both forms
        s3, p3 = G.config3()
        rec["batched"] = {"workload": "config3: 256 scenes, rooms U(3,10)xU(3,8)xU(2.5,4) m, Sabine orders "
                                      "6-18, 1-8 s at 16 kHz, lines and circles, tiers, T=64"}
        for fd in (args.fd, other):
            rec["batched"][fd] = measure_batched(s3, with_fd(p3, fd), nfb, torch)
        del s3
        rec["differentiation"] = {"workload": "config4: 32 scenes, 6x5x3 m, K=10 (1561 images), 2 s at 16 kHz, "
                                              "8-knot source paths, tiers, T=64; batched forward + backward "
                                              "(dL/dx, dL/dbeta_w, dL/dknots)"}
        for fd in (args.fd, other):
            rec["differentiation"][fd] = measure_differentiation(fd, 3, torch)

    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(scenes, par0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
