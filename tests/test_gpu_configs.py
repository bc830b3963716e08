"""GPU parity at the full sizes of the differentiation and large workloads, in
the launch configuration the benchmark times, on outputs the FP64 oracle can
evaluate one by one (its output-subset mode solves the delays it needs locally).

* 32-scene differentiation workload (6x5x3 m, K = 10, 2 s, 8-knot paths): the
  batched forward of all scenes, checked on sampled outputs of two scenes; the
  backward of all scenes for a loss whose gradient dL/dy is non-zero only on
  sampled outputs of scenes 0-3, so the oracle's adjoints and its FP64 central
  differences (step 1e-6) for the knots and the wall coefficients of those four
  scenes stay cheap.  Scenes with dL/dy = 0 must get exactly zero gradients.
* the large workload (64 scenes of 12x9x4 m, 48 kHz, 10 s, moving source and
  receiver, 8-mic array, K = 20 -> 11 521 images, T = 96): the batched forward
  of all 64 scenes (one persistent launch, graph-replayed), checked on sampled
  outputs of 4 scenes x 8 mics; the batched backward of all 64 scenes for a loss
  whose gradient is non-zero on a few outputs of scenes 0 and 5: dL/dbeta
  against the oracle, dL/dx against its exact transpose, the knots against FP64
  central differences, and exactly zero for every other scene."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_03065_amd import scenegen as G

pytestmark = pytest.mark.gpu

FORMS = {"table": 0, "farrow": 1}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def config4_case():
    scenes, par = G.config4()
    rng = np.random.default_rng(44)
    sparse = {}
    for s in range(4):
        idx = np.sort(rng.choice(scenes[s].n_out, 48, replace=False))
        sparse[s] = (idx, rng.standard_normal((scenes[s].n_mics, 48)))
    # FP64 central differences (step 1e-6) of L = <gy, y> in the source knots and
    # the wall coefficients of scenes 0-3 (the oracle's output-subset mode)
    h = 1e-6
    fd_knots, fd_beta = {}, {}
    for s in range(4):
        sc = scenes[s]
        idx, w = sparse[s]
        loss = lambda c: np.sum(O.forward(c, par, idx=idx) * w)
        g = np.zeros_like(sc.src.p)
        for k in range(sc.src.p.shape[0]):
            for a in range(3):
                sp, sm = sc.copy(), sc.copy()
                sp.src.p[k, a] += h
                sm.src.p[k, a] -= h
                g[k, a] = (loss(sp) - loss(sm)) / (2 * h)
        fd_knots[s] = g
        b = np.zeros(6)
        for wall in range(6):
            sp, sm = sc.copy(), sc.copy()
            sp.beta = sc.beta.copy()
            sm.beta = sc.beta.copy()
            sp.beta[wall] += h
            sm.beta[wall] -= h
            b[wall] = (loss(sp) - loss(sm)) / (2 * h)
        fd_beta[s] = b
    return scenes, par, sparse, (fd_knots, fd_beta)


@pytest.mark.parametrize("form", sorted(FORMS))
def test_config4_batched_forward_and_gradients(torch_cuda, config4_case, form):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par0, sparse, fd = config4_case
    par = dataclasses.replace(par0, fd_kind=FORMS[form])
    print("config4:", form, "32 scenes, batched forward + backward", flush=True)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward_batched(x, graph=True)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    ys = plan.unpack_y(y)
    rng = np.random.default_rng(4)
    for s in (0, 21):
        idx = np.sort(rng.choice(scenes[s].n_out, 96, replace=False))
        assert rel(ys[s][:, idx].cpu().numpy(), O.forward(scenes[s], par0, idx=idx)) <= 1e-5, s

    gy_full = np.zeros(plan.y_total, np.float32)
    dense = {}
    for s, (idx, w) in sparse.items():
        g = np.zeros((scenes[s].n_mics, scenes[s].n_out))
        g[:, idx] = w
        dense[s] = g
        gy_full[plan.y_off[s]:plan.y_off[s] + g.size] = g.reshape(-1)
    gx, gb, gs = plan.backward(x, torch.from_numpy(gy_full).cuda(), batched=True)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    gx, gb, gs = gx.cpu().numpy(), gb.cpu().numpy(), gs.cpu().numpy()
    fd_knots, fd_beta = fd
    for s in range(4):
        assert rel(gb[s], O.grad_beta(scenes[s], par0, dense[s])) <= 1e-4, s
        assert rel(gb[s], fd_beta[s]) <= 1e-3, s
        o = plan.x_off[s]
        assert rel(gx[o:o + scenes[s].n_in], O.adjoint_x(scenes[s], par0, dense[s])) <= 1e-5, s
        k0 = plan.src_off[s]
        assert rel(gs[k0:k0 + scenes[s].src.p.shape[0]], fd_knots[s]) <= 1e-3, s
    # scenes without loss gradient get exactly zero
    assert not np.any(gb[4:])
    assert not np.any(gx[plan.x_off[4]:])
    assert not np.any(gs[plan.src_off[4]:])


@pytest.fixture(scope="module")
def config5_case():
    scenes, par = G.config5()
    rng = np.random.default_rng(55)
    check = (0, 21, 42, 63)
    idx = {s: np.sort(rng.choice(scenes[s].n_out, 8, replace=False)) for s in check}
    ref = {s: O.forward(scenes[s], par, idx=idx[s]) for s in check}
    sparse, dense = {}, {}
    for s in (0, 5):
        ii = np.sort(rng.choice(scenes[s].n_out - 2000, 6, replace=False)) + 1000
        sparse[s] = (ii, rng.standard_normal((scenes[s].n_mics, 6)))
        g = np.zeros((scenes[s].n_mics, scenes[s].n_out))
        g[:, ii] = sparse[s][1]
        dense[s] = g
    gb = {s: O.grad_beta(scenes[s], par, dense[s]) for s in (0, 5)}
    gx0 = O.adjoint_x(scenes[0], par, dense[0])
    sc = scenes[0]
    ii, w = sparse[0]
    fd = np.zeros_like(sc.src.p)
    h = 1e-6
    for k in range(sc.src.p.shape[0]):
        for a in range(3):
            sp, sm = sc.copy(), sc.copy()
            sp.src.p[k, a] += h
            sm.src.p[k, a] -= h
            fd[k, a] = (np.sum(O.forward(sp, par, idx=ii) * w) - np.sum(O.forward(sm, par, idx=ii) * w)) / (2 * h)
    return scenes, par, idx, ref, dense, gb, gx0, fd


@pytest.mark.parametrize("form", sorted(FORMS))
def test_config5_batched_forward_and_gradients(torch_cuda, config5_case, form):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par0, idx, ref, dense, gb_ref, gx0_ref, fd = config5_case
    par = dataclasses.replace(par0, fd_kind=FORMS[form])
    print("config5:", form, "64 scenes x 8 mics, K=20, 48 kHz, 10 s: batched forward + backward", flush=True)
    plan = Plan(scenes, par)
    assert all(int(n) == 11521 for n in plan.n_images)
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward_batched(x, graph=True)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    ys = plan.unpack_y(y)
    for s, ii in idx.items():
        assert rel(ys[s][:, ii].cpu().numpy(), ref[s]) <= 1e-5, s
    del y, ys
    gy = torch.zeros(plan.y_total, dtype=torch.float32, device="cuda")
    for s, g in dense.items():
        gy[plan.y_off[s]:plan.y_off[s] + g.size] = torch.from_numpy(g.reshape(-1).astype(np.float32)).cuda()
    print("config5:", form, "batched backward", flush=True)
    gx, gb, gs = plan.backward(x, gy, batched=True, graph=True)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    gx, gb, gs = gx.cpu().numpy(), gb.cpu().numpy(), gs.cpu().numpy()
    for s in (0, 5):
        assert rel(gb[s], gb_ref[s]) <= 1e-4, s
    assert rel(gx[plan.x_off[0]:plan.x_off[0] + scenes[0].n_in], gx0_ref) <= 1e-5
    k0 = scenes[0].src.p.shape[0]
    assert rel(gs[:k0], fd) <= 1e-3
    others = [s for s in range(len(scenes)) if s not in (0, 5)]
    assert not np.any(gb[others])
    assert not np.any(gx[plan.x_off[1]:plan.x_off[5]]) and not np.any(gx[plan.x_off[6]:])
    assert not np.any(gs[plan.src_off[6]:])
