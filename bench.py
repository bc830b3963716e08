"""Throughput of the moving image-source synthesis on one MI355X.

Headline workload: the large batched configuration (64 scenes of a 12x9x4 m
room, 48 kHz, 10 s sources, moving source and receiver, 8-mic circular array,
every image up to order 20 (11521 per scene), tiers 48 k / 3 k / 300 Hz, 96-tap
sinc).  A step is one batched forward (one persistent launch per kernel, replayed
from a HIP graph) over a batch of --scenes of those 64 scenes with the source
signals already in HBM; a whole 64-scene batch takes about 16 such steps, longer
than the driver's 20 timed steps allow.  Prints one JSON line.

Metric: image-sample taps/s = sum over scenes, mics, images of (n_in + T - 1) * T
taps per step / seconds per step.  Forward+backward counts four tap chains per
forward tap (forward, dL/dx, and the value and derivative chains of the gain and
delay adjoints).  The Farrow form computes the same output (within the same
tolerance) without visiting every tap; its rate is quoted in the same
equivalent taps/s, and its kernel rooflines count the work it really does.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2508_03065_amd import scenegen as G  # noqa: E402

PEAK_FP32 = 157.3e12      # MI355X FP32 vector, FLOP/s
PEAK_LDS = 256 * 256 * 2.4e9   # LDS reads, B/s: 256 CUs x 256 B/clk (b128) x 2.4 GHz

# Algorithmic flops per tap (table form) or per image sample (Farrow form, order M).
FLOPS_PER_TAP = 4             # forward, dL/dx: the interpolated coefficient and the multiply-add (2 FMAs)
FLOPS_PER_TAP_GD = 8          # gain/delay adjoint: the value and the derivative chains


def table_lds_per_tap(outputs_per_lane: int, taps: int) -> float:
    """Table form, LDS bytes per tap: the source sample and the row's two FP32
    quadratic-table values (12 B), and its FP16 second difference (2 B) on the tap
    quads that carry one (3/4 of the half-width for up to 64 taps, half of it for
    96 and 128); with two adjacent outputs per lane one table read and one new
    source quad serve both outputs' taps."""
    quads = taps // 8
    with_d2 = taps // 16 if taps >= 96 else taps // 8 - taps // 32
    return (12.0 + 2.0 * with_d2 / quads) / outputs_per_lane


def farrow_lds_per_sample(order: int) -> int:
    """Farrow form: the M+1 filtered values read per image sample (40 B for M <= 9)."""
    return 40 if order <= 9 else 48


def farrow_flops(order: int) -> dict:
    """Farrow form, per image sample: forward = Horner of degree M (M FMAs), the cubic
    delay offset (3 FMAs), the gain times the polynomial added to the output (1 FMA);
    dL/dx gather = the M+1 sums u_k += (gy g) s^k and the M powers of s; gain/delay
    adjoint = Horner for the value and its derivative (2M FMAs), the delay offset
    (3) and the dL/dbeta_i and dL/dD products (3)."""
    return {"fwd": 2 * (order + 4), "adjx": 2 * (2 * order + 1), "adjp": 2 * (2 * order + 6)}


WORKLOADS = {
    "config5": ("large batched: 12x9x4 m room, 48 kHz, 10 s, moving source and receiver (PWL, <= 2 m/s), "
                "8-mic circular array r=5 cm, K=20 (11521 images), tiers 48k/3k/300 Hz, T=96", G.config5),
    "config2": ("paper-scale plain: 8x6x3.5 m room, K=12 (2625 images), 4 s at 16 kHz, "
                "tiers 16k/1k/100 Hz, T=64, 1 mic", G.config2),
}
FD_KINDS = {"table": 0, "farrow": 1}
KERNEL_OF = {"table": {"fwd": ("k_synth", "msim_kernels.hip"), "adjx": ("k_adjx", "msim_adjoint.hip"),
                       "adjp": ("k_adjp", "msim_adjoint.hip")},
             "farrow": {"fwd": ("k_farrow", "msim_farrow.hip"), "adjx": ("k_farrow_u", "msim_farrow.hip"),
                        "adjp": ("k_farrow_gd", "msim_farrow.hip")}}
PROFILE_KEY = {"fwd": "synth", "adjx": "adjx", "adjp": "adjp"}


def with_fd(par, fd: str):
    return dataclasses.replace(par, fd_kind=FD_KINDS[fd])


def source_sha(fname: str) -> str:
    h = hashlib.sha256()
    for f in (fname, "msim_device.h", "msim_internal.h"):
        with open(os.path.join(ROOT, "paper_2508_03065_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_traffic(kernel: str, workload: str, src: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>__<workload>__hbm_pmc.md (FETCH_SIZE and WRITE_SIZE, scaled by
    the copy-kernel factors recorded there), or None when there is none or the
    kernel's sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s__%s__hbm_pmc.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    tb = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not sha or not tb or sha.group(1) != source_sha(src):
        return None
    return float(tb.group(1))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_SAMPLE = """
import sys, time, json, numpy as np
sys.path.insert(0, {root!r})
from oracle import oracle as O
from paper_2508_03065_amd import scenegen as G
scenes, par = G.{gen}(n_scenes=1) if {gen!r} == "config5" else G.{gen}()
sc = scenes[0]
idx = np.sort(np.random.default_rng(7).choice(sc.n_out, {n}, replace=False))
t0 = time.perf_counter()
O.forward(sc, par, idx=idx)
print(json.dumps({{"s": time.perf_counter() - t0}}))
"""


def cpu_baseline(workload: str, scenes, par, target_s: float = 15.0):
    """The FP64 oracle on the host cores, on a bounded sample of output samples
    of the first scene (tier-emulating mode, every image, exact kernel), and the
    same on one core in a child process (OMP_NUM_THREADS=1) on a smaller sample."""
    from oracle import oracle as O
    sc = scenes[0]
    rng = np.random.default_rng(123)
    n_img = O.count_images(sc.max_order)
    n, dt = 16, 0.0
    while True:
        idx = np.sort(rng.choice(sc.n_out, n, replace=False))
        t0 = time.perf_counter()
        O.forward(sc, par, idx=idx)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * target_s or n >= sc.n_out:
            break
        n = int(min(sc.n_out, max(2 * n, n * target_s / max(dt, 1e-3))))
    per_out = float(sc.n_mics) * n_img * par.taps
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    out = {"value": n * per_out / dt, "unit": "taps/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "%d random output samples x %d mics x %d images x %d taps of the first scene "
                     "(FP64, exact kernel, tier-emulating delays), %.1f s" % (n, sc.n_mics, n_img, par.taps, dt)}
    n1 = max(4, int(n / max(cores, 1) / 2))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    gen = WORKLOADS[workload][1].__name__
    try:
        r = subprocess.run([sys.executable, "-c", _ORACLE_SAMPLE.format(root=ROOT, gen=gen, n=n1)], env=env,
                           capture_output=True, text=True, timeout=300)
        s1 = json.loads(r.stdout.strip().splitlines()[-1])["s"]
        out["one_core"] = {"value": n1 * per_out / s1, "unit": "taps/s", "cores": 1,
                           "sample": "%d random output samples of the same scene, %.1f s" % (n1, s1)}
    except Exception as e:  # the one-core figure is context only
        out["one_core"] = {"error": str(e)[:200]}
    return out


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def kernel_roofline(fd, kind, prof, work_flops, workload, lds_bytes=None, gather=False):
    """Roofline of one kernel kind from the plan's HIP-event profile: achieved
    FLOP/s = algorithmic flops per launch / average launch duration."""
    kernel, src = KERNEL_OF["farrow" if kind == "adjx" and gather else fd][kind]
    if fd == "table" and kind == "adjx" and gather:
        workload += "_table"          # the gather over the table form's delay groups
    key = PROFILE_KEY[kind]
    n = max(1, prof[key + "_launches"])
    kms = prof[key + "_ms"] / n
    achieved = work_flops / (kms * 1e-3)
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
           "frac": achieved / PEAK_FP32, "traffic": pmc_traffic(kernel, workload, src), "kernel": kernel,
           "kernel_ms": kms, "flops_per_launch": work_flops}
    if lds_bytes is not None:
        out["lds"] = {"achieved": lds_bytes / (kms * 1e-3) / 1e12, "peak": PEAK_LDS / 1e12, "unit": "TB/s",
                      "frac": lds_bytes / (kms * 1e-3) / PEAK_LDS, "bytes_per_launch": lds_bytes}
    return out


def image_samples(plan, par):
    return plan.forward_taps / par.taps


def fwd_work(plan, par, fd):
    if fd == "table":
        t = plan.forward_taps
        return t * FLOPS_PER_TAP, t * table_lds_per_tap(plan.tuning()["outputs_per_lane"], par.taps)
    s = image_samples(plan, par)
    return s * farrow_flops(par.farrow_order)["fwd"], s * farrow_lds_per_sample(par.farrow_order)


def bwd_work(plan, par, fd):
    """Algorithmic flops of one launch of the dL/dx kernel (the table form's own
    transpose, or the Farrow gather that both forms use by default) and of the
    gain/delay kernel."""
    s = image_samples(plan, par)
    f = farrow_flops(par.farrow_order)
    t = plan.forward_taps
    adjx = s * f["adjx"] if plan.tuning()["adjx_gather"] else t * FLOPS_PER_TAP
    return {"adjx": adjx, "adjp": t * FLOPS_PER_TAP_GD if fd == "table" else s * f["adjp"]}


def measure_batched_form(scenes, par, fd, steps, warmup, fb_steps, torch, workload):
    """Batched forward (graph replays) and forward+backward of one plan, with
    rooflines of its kernels from a profiled pass without the graph."""
    from paper_2508_03065_amd.msim import Plan
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        plan.forward_batched(x, y)
    torch.cuda.synchronize()
    if plan.device_status() != 0:
        raise RuntimeError("device status flags set")
    sec = timed(lambda: plan.forward_batched(x, y), steps, torch)
    plan.profile_begin()
    timed(lambda: plan.forward_batched(x, y, graph=False), 1, torch)
    pf = plan.profile_end()
    flops, lds = fwd_work(plan, par, fd)
    taps = plan.forward_taps
    rec = {"value": taps / sec, "unit": "taps/s", "ms_per_step": sec * 1e3, "steps": steps,
           "scenes": len(scenes), "images": int(plan.n_images.sum()), "taps_per_step": taps,
           "outputs_per_lane": plan.tuning()["outputs_per_lane"],
           "phases_ms_per_step": {k[:-3]: pf[k] for k in ("synth_ms", "reduce_ms", "filter_ms")},
           "roofline": kernel_roofline(fd, "fwd", pf, flops, workload, lds)}
    # forward + backward: dense dL/dy, every gradient (x, the walls, the source knots)
    g = torch.Generator().manual_seed(5)
    gy = torch.randn(plan.y_total, generator=g).cuda()
    plan.backward(x, gy, batched=True)
    out = plan.last_backward_buffers

    def fwd_bwd():
        plan.forward_batched(x, y)
        plan.backward(x, gy, batched=True, out=out)
    fwd_bwd()
    sfb = timed(fwd_bwd, fb_steps, torch)
    plan.profile_begin()
    plan.forward_batched(x, y, graph=False)
    plan.backward(x, gy, batched=True, graph=False, out=out)
    torch.cuda.synchronize()
    pb = plan.profile_end()
    bw = bwd_work(plan, par, fd)
    kern = sum(pb[k] for k in ("synth_ms", "reduce_ms", "adjx_ms", "adjp_ms", "params_ms", "filter_ms"))
    step_flops = flops + bw["adjx"] + bw["adjp"]
    rec["fwd_bwd"] = {
        "value": 4 * taps / sfb, "unit": "taps/s", "ms_per_step": sfb * 1e3, "steps": fb_steps,
        "phases_ms_per_step": {k[:-3]: pb[k] for k in
                               ("synth_ms", "reduce_ms", "adjx_ms", "adjp_ms", "params_ms", "filter_ms")},
        "roofline": {"bound": "alu", "achieved": step_flops / (kern * 1e-3) / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": step_flops / (kern * 1e-3) / PEAK_FP32,
                     "flops_per_step": step_flops, "kernel_ms_per_step": kern,
                     "kernels": {"adjx": kernel_roofline(fd, "adjx", pb, bw["adjx"], workload,
                                                         gather=bool(plan.tuning()["adjx_gather"])),
                                 "adjp": kernel_roofline(fd, "adjp", pb, bw["adjp"], workload)}}}
    del plan, x, y, gy, out
    torch.cuda.empty_cache()
    return rec


def measure_full_batch(scenes, par, steps, torch):
    """Batched forward of every scene of the workload in one launch (graph replays)."""
    from paper_2508_03065_amd.msim import Plan
    t0 = time.perf_counter()
    plan = Plan(scenes, par)
    t_plan = time.perf_counter() - t0
    x = plan.pack_x([s.x for s in scenes])
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
    plan.forward_batched(x, y)
    sec = timed(lambda: plan.forward_batched(x, y), steps, torch)
    out = {"fd": "farrow", "scenes": len(scenes), "images": int(plan.n_images.sum()), "steps": steps,
           "taps_per_step": plan.forward_taps, "value": plan.forward_taps / sec, "unit": "taps/s",
           "ms_per_step": sec * 1e3, "plan_s": t_plan}
    del plan, x, y
    torch.cuda.empty_cache()
    return out


def measure_batched_vs_plain(scenes, par, steps, torch, with_backward):
    """Seconds per step of the batched path (graph replays) and of the plain
    path (launches per scene) on the same plan."""
    from paper_2508_03065_amd.msim import Plan
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
    out = {"scenes": len(scenes), "images": int(plan.n_images.sum())}
    if with_backward:
        gy = torch.randn(plan.y_total, generator=torch.Generator().manual_seed(4)).cuda()
        plan.backward(x, gy, batched=True)
        bufs = plan.last_backward_buffers
        plan.backward(x, gy)
        pbufs = plan.last_backward_buffers

        def b():
            plan.forward_batched(x, y)
            plan.backward(x, gy, batched=True, out=bufs)

        def p():
            plan.forward(x, y)
            plan.backward(x, gy, out=pbufs)
        taps = 4 * plan.forward_taps
    else:
        def b():
            plan.forward_batched(x, y)

        def p():
            plan.forward(x, y)
        taps = plan.forward_taps
    b()
    p()
    sb = timed(b, steps, torch)
    sp = timed(p, steps, torch)
    out.update({"taps_per_step": taps, "value": taps / sb, "unit": "taps/s", "ms_per_step": sb * 1e3,
                "plain_value": taps / sp, "plain_ms_per_step": sp * 1e3, "speedup_vs_plain": sp / sb})
    del plan, x, y
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config5", choices=sorted(WORKLOADS))
    ap.add_argument("--scenes", type=int, default=4, help="scenes per step (config5: a batch of its 64 scenes)")
    ap.add_argument("--fd", default="table", choices=sorted(FD_KINDS),
                    help="fractional-delay form of the headline measurement (the other is reported beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="the headline form only: its forward and forward+backward (no other form or workload)")
    ap.add_argument("--fwd-only", action="store_true", help="with --no-extra: the forward only")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB: the reference kernel that "
                         "scales the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(scenes or output tiles would shard with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    t_start = time.perf_counter()

    def note(msg):
        print("[bench %6.1f s] %s" % (time.perf_counter() - t_start, msg), file=sys.stderr, flush=True)

    desc, gen = WORKLOADS[args.workload]
    if args.workload == "config5":
        all_scenes, par0 = gen(n_scenes=max(args.scenes, 1))
    else:
        all_scenes, par0 = gen()
    scenes = all_scenes[: args.scenes]
    other = "farrow" if args.fd == "table" else "table"
    fb_steps = max(1, args.steps // 10)

    note("headline: %s, %d scenes, %s form" % (args.workload, len(scenes), args.fd))
    from paper_2508_03065_amd.msim import Plan
    par = with_fd(par0, args.fd)
    if args.fwd_only:
        plan = Plan(scenes, par)
        x = plan.pack_x([s.x for s in scenes])
        y = torch.empty(plan.y_total, dtype=torch.float32, device="cuda")
        for _ in range(args.warmup):
            plan.forward_batched(x, y)
        sec = timed(lambda: plan.forward_batched(x, y), args.steps, torch)
        plan.profile_begin()
        timed(lambda: plan.forward_batched(x, y, graph=False), 1, torch)
        pf = plan.profile_end()
        flops, lds = fwd_work(plan, par, args.fd)
        head = {"value": plan.forward_taps / sec, "ms_per_step": sec * 1e3, "images": int(plan.n_images.sum()),
                "taps_per_step": plan.forward_taps, "outputs_per_lane": plan.tuning()["outputs_per_lane"],
                "roofline": kernel_roofline(args.fd, "fwd", pf, flops, args.workload, lds),
                "phases_ms_per_step": {k[:-3]: pf[k] for k in ("synth_ms", "reduce_ms", "filter_ms")}}
        del plan, x, y
        torch.cuda.empty_cache()
    else:
        head = measure_batched_form(scenes, par, args.fd, args.steps, args.warmup, fb_steps, torch, args.workload)
    rec = {
        "metric": "image-sample taps/s (batched forward, %s form of the fractional delay)" % args.fd,
        "value": head["value"],
        "unit": "taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded N(0,1) sources, seeded trajectories and walls)",
        "config": {"workload": args.workload + ": " + desc, "fd": args.fd, "scenes_per_step": len(scenes),
                   "scenes_in_workload": 64 if args.workload == "config5" else len(all_scenes),
                   "images": head["images"], "taps_per_step": head["taps_per_step"],
                   "outputs_per_lane": head["outputs_per_lane"]},
        "phases_ms_per_step": head["phases_ms_per_step"],
        "roofline": head["roofline"],
    }
    if "fwd_bwd" in head:
        rec["fwd_bwd"] = head["fwd_bwd"]

    if not args.no_extra:
        note("other form: %s" % other)
        rec[other] = measure_batched_form(scenes, with_fd(par0, other), other, max(3, args.steps // 4), 1,
                                          fb_steps, torch, args.workload)
        del all_scenes, scenes
        if args.workload == "config5":
            # the whole 64-scene batch as one launch, in the faster form
            note("all 64 scenes, farrow form")
            s64, p64 = G.config5()
            rec["full_batch"] = measure_full_batch(s64, with_fd(p64, "farrow"), 2, torch)
            del s64
        note("batched vs plain: config4 forward+backward")
        s4, p4 = G.config4()
        rec["batched_vs_plain"] = {
            "config4_fwd_bwd": {"workload": "config4: 32 scenes, 6x5x3 m, K=10 (1561 images), 2 s at 16 kHz, "
                                            "8-knot source paths, tiers, T=64; forward + backward (dL/dx, "
                                            "dL/dbeta_w, dL/dknots)"}}
        for fd in ("table", "farrow"):
            rec["batched_vs_plain"]["config4_fwd_bwd"][fd] = measure_batched_vs_plain(
                s4, with_fd(p4, fd), max(2, args.steps // 5), torch, True)
        del s4
        note("batched vs plain: config3 forward")
        s3, p3 = G.config3()
        rec["batched_vs_plain"]["config3_fwd"] = {
            "workload": "config3: 256 scenes, rooms U(3,10)xU(3,8)xU(2.5,4) m, Sabine orders 6-18, "
                        "1-8 s at 16 kHz, lines and circles, tiers, T=64"}
        for fd in ("table", "farrow"):
            rec["batched_vs_plain"]["config3_fwd"][fd] = measure_batched_vs_plain(
                s3, with_fd(p3, fd), max(2, args.steps // 5), torch, False)
        del s3

    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        note("cpu baseline")
        cs, cp = (G.config5(n_scenes=1) if args.workload == "config5" else G.config2())
        rec["cpu_baseline"] = cpu_baseline(args.workload, cs, cp)
    note("done")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
