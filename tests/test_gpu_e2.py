"""GPU parity on the paper-style data front-end: rooms with a 15 cm mic pair,
band-limited random source paths (dense knots: 8 per second) mixed 1:10 with
static sources, through the batched forward of both fractional-delay forms,
and the backward (dL/dx, dL/dbeta, dL/dknots) against the FP64 oracle."""
import dataclasses

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
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("form", [0, 1])
def test_e2_batched_forward(torch_cuda, form):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par0, labels = G.e2_scenes(seed=8, n_scenes=12, seconds=1.0, max_order=6)
    par = dataclasses.replace(par0, fd_kind=form)
    print("e2 scenes, form", form, labels, flush=True)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward_batched(x, graph=True)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    ys = plan.unpack_y(y)
    rng = np.random.default_rng(9)
    for s in (0, 1, 5, 11):
        idx = np.sort(rng.choice(scenes[s].n_out, 80, replace=False))
        assert rel(ys[s][:, idx].cpu().numpy(), O.forward(scenes[s], par0, idx=idx)) <= 1e-5, s


def test_e2_backward(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    scenes, par0, _ = G.e2_scenes(seed=10, n_scenes=2, seconds=0.5, max_order=4)
    sc = scenes[1]                                   # a band-limited moving source, 9 knots
    assert sc.src.p.shape[0] > 2
    par = dataclasses.replace(par0, fd_kind=1)
    plan = Plan([sc], par)
    x = plan.pack_x([sc.x])
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(sc.n_out, 40, replace=False))
    gy = np.zeros((sc.n_mics, sc.n_out))
    gy[:, idx] = rng.standard_normal((sc.n_mics, 40))
    gx, gb, gs = plan.backward(x, torch.from_numpy(gy.reshape(-1).astype(np.float32)).cuda())
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert rel(gx.cpu().numpy(), O.adjoint_x(sc, par0, gy)) <= 1e-5
    assert rel(gb.cpu().numpy()[0], O.grad_beta(sc, par0, gy)) <= 1e-4
    fd = np.zeros_like(sc.src.p)
    for k in range(sc.src.p.shape[0]):
        for a in range(3):
            sp, sm = sc.copy(), sc.copy()
            sp.src.p[k, a] += 1e-6
            sm.src.p[k, a] -= 1e-6
            fd[k, a] = (np.sum(O.forward(sp, par0, idx=idx) * gy[:, idx]) -
                        np.sum(O.forward(sm, par0, idx=idx) * gy[:, idx])) / 2e-6
    assert rel(gs.cpu().numpy(), fd) <= 1e-3
