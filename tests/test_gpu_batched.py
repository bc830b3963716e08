"""GPU tests of the batched forward: one persistent ticket-scheduled launch over
every scene, replayed from a HIP graph, and the autotuner that picks its launch
shape.  It must equal the plain per-scene path bit for bit and the FP64 oracle to
relative L2 <= 1e-5."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_03065_amd import scenegen as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def mixed_scenes(n=9, taps=64):
    out = []
    par = None
    for s in range(n):
        sc, par = G.small_scene(seed=100 + s, max_order=2 + s % 5, seconds=0.03 + 0.02 * (s % 4), taps=taps,
                                n_mics=1 + s % 3, circle=(s % 3 == 1), moving_rcv=(s % 4 == 3))
        out.append(sc)
    return out, par


def test_batched_equals_plain_and_oracle(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par = mixed_scenes()
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y_plain = plan.forward(x).clone()
    y_direct = plan.forward_batched(x, graph=False).clone()
    y_graph = plan.forward_batched(x, graph=True).clone()
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert torch.equal(y_plain, y_direct)
    assert torch.equal(y_plain, y_graph)
    for s, yv in enumerate(plan.unpack_y(y_graph)):
        assert rel(yv.cpu().numpy(), O.forward(scenes[s], par)) <= 1e-5


def test_graph_replays_with_eager_work_between(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par = mixed_scenes(5, taps=32)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    ref = plan.forward(x).clone()
    y = torch.empty_like(ref)
    for r in range(4):
        y.fill_(float(r + 1))                       # eager work on the same buffers between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        plan.forward_batched(x, y, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), r
        assert torch.isfinite(junk)


def test_autotune_keeps_result(torch_cuda, tmp_path):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par = mixed_scenes(7)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    cache = str(tmp_path / "tune.jsonl")
    best = plan.autotune(x, cache_path=cache)
    assert best["threads"] in (512, 1024) and best["ms"] > 0
    assert os.path.exists(cache)
    again = Plan(scenes, par).autotune(x, cache_path=cache)     # read back from the cache
    assert (again["threads"], again["group_cap"]) == (best["threads"], best["group_cap"])
    y_b = plan.forward_batched(x).clone()
    y_p = plan.forward(x).clone()
    torch.cuda.synchronize()
    assert torch.equal(y_b, y_p)
    for s, yv in enumerate(plan.unpack_y(y_b)):
        assert rel(yv.cpu().numpy(), O.forward(scenes[s], par)) <= 1e-5


@pytest.mark.parametrize("threads,cap", [(512, 0), (1024, 64), (512, 256)])
def test_launch_shapes(torch_cuda, threads, cap):
    from paper_2508_03065_amd.msim import Plan
    scenes, par = mixed_scenes(4)
    plan = Plan(scenes, par)
    plan.set_tuning(threads, cap)
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward_batched(x)
    for s, yv in enumerate(plan.unpack_y(y)):
        assert rel(yv.cpu().numpy(), O.forward(scenes[s], par)) <= 1e-5


def test_config3_sampled(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par = G.config3()
    print("config3: 256 scenes, Sabine orders, lines and circles", flush=True)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward_batched(x)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    ys = plan.unpack_y(y)
    rng = np.random.default_rng(5)
    for s in (0, 1, 97, 255):
        idx = np.sort(rng.choice(scenes[s].n_out, 60, replace=False))
        assert rel(ys[s][:, idx].cpu().numpy(), O.forward(scenes[s], par, idx=idx)) <= 1e-5, s


@pytest.mark.parametrize("fd", [0, 1])
def test_backward_batched_equals_plain(torch_cuda, fd):
    """The batched backward (one persistent launch per kernel over every scene,
    direct and graph-replayed, with eager work between the replays) equals the
    plain per-scene backward bit for bit, for both fractional-delay forms."""
    import dataclasses
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par = mixed_scenes(6)
    par = dataclasses.replace(par, fd_kind=fd)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    gy = torch.randn(plan.y_total, generator=torch.Generator().manual_seed(9)).cuda()
    ref = [t.clone() for t in plan.backward(x, gy)]
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    for graph in (False, True, True, True):
        junk = torch.randn(1 << 16, device="cuda").sum()
        got = plan.backward(x, gy, batched=True, graph=graph)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), graph
        assert torch.isfinite(junk)
    assert plan.device_status() == 0


def test_autotune_corrupt_cache_falls_back_to_timing(torch_cuda, tmp_path):
    """Malformed lines, and a line for this plan with a shape it refuses, are
    passed over: the tuner times the candidates, applies the best, appends a
    good line, and a plan that then reads the cache takes that line."""
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par = mixed_scenes(5)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    cache = tmp_path / "tune.jsonl"
    with open(cache, "w") as f:
        f.write('{"key": "gfx950/F0/M9/T64\n')                     # truncated
        f.write("not json at all\n")
        f.write('{"key": 5, "threads": "many"}\n')
    # the plan's own key with a shape outside the allowed set, and one it refuses
    key_probe = Plan(scenes, par).autotune(x, cache_path=str(tmp_path / "probe.jsonl"))
    lines = open(tmp_path / "probe.jsonl").read().splitlines()
    key = lines[-1].split('"key": "')[1].split('"')[0]
    with open(cache, "a") as f:
        f.write('{"key": "%s", "threads": 7, "group_cap": 0, "outputs_per_lane": 1, "ms": 1.0}\n' % key)
        f.write('{"key": "%s", "threads": 512, "group_cap": 0, "outputs_per_lane": 4, "ms": 1.0}\n' % key)
    before = open(cache).read()
    best = plan.autotune(x, cache_path=str(cache))
    assert best["ms"] > 0                                   # timed, not read
    after = open(cache).read()
    assert after.startswith(before) and after.count("\n") == before.count("\n") + 1
    again = Plan(scenes, par).autotune(x, cache_path=str(cache))
    assert (again["threads"], again["group_cap"], again["outputs_per_lane"]) == \
        (best["threads"], best["group_cap"], best["outputs_per_lane"])
    assert key_probe["threads"] in (512, 1024)
    y = plan.forward_batched(x)
    torch.cuda.synchronize()
    for s, yv in enumerate(plan.unpack_y(y)):
        assert rel(yv.cpu().numpy(), O.forward(scenes[s], par)) <= 1e-5


@pytest.mark.parametrize("fd", [0, 1])
def test_large_groups_forward_and_backward(torch_cuda, fd):
    """Delay groups up to 512 images (more than one LDS chunk of image
    descriptors in every kernel that stages them): forward, dL/dx and dL/dbeta
    against the oracle, in the batched launch."""
    import dataclasses
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    a, par = G.small_scene(seed=131, max_order=7, seconds=0.05, taps=64, n_mics=2)
    b, _ = G.small_scene(seed=132, max_order=6, seconds=0.04, taps=64, moving_rcv=True)
    scenes = [a, b]
    par = dataclasses.replace(par, fd_kind=fd)
    plan = Plan(scenes, par)
    plan.set_tuning(1024, 512)
    print("large groups, fd", fd, flush=True)
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward_batched(x)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    for s, yv in enumerate(plan.unpack_y(y)):
        assert rel(yv.cpu().numpy(), O.forward(scenes[s], par)) <= 1e-5, s
    rng = np.random.default_rng(17)
    gys = [rng.standard_normal((s.n_mics, s.n_out)) for s in scenes]
    gy = torch.from_numpy(np.concatenate([g.reshape(-1) for g in gys]).astype(np.float32)).cuda()
    gx, gb, _ = plan.backward(x, gy, batched=True, want_src=False)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    gx, gb = gx.cpu().numpy(), gb.cpu().numpy()
    for s, sc in enumerate(scenes):
        o = plan.x_off[s]
        assert rel(gx[o:o + sc.n_in], O.adjoint_x(sc, par, gys[s])) <= 1e-5, s
        assert rel(gb[s], O.grad_beta(sc, par, gys[s])) <= 1e-4, s
