"""GPU parity of the adjoint of the Farrow form (MSIM_FD_FARROW, Sec. II-B
Eq. 3-5) through the C-ABI: dL/dx is the transposed filter bank applied to the
gathered sums u_k, dL/dbeta and dL/dD use the polynomial's value and
derivative in the fractional delay.  Against the FP64 oracle's exact kernel:
the exact transpose for dL/dx, the analytic dL/dbeta, and FP64 central finite
differences for the source knots, at the same bars as the table form."""
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


def farrow(par, order=9):
    return dataclasses.replace(par, fd_kind=1, farrow_order=order)


def gpu_backward(scenes, par, gys, torch):
    from paper_2508_03065_amd.msim import Plan
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    gy = torch.from_numpy(np.concatenate([g.reshape(-1) for g in gys]).astype(np.float32)).cuda()
    gx, gb, gs = plan.backward(x, gy)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, gx.cpu().numpy(), gb.cpu().numpy(), gs.cpu().numpy()


def fd_knots(sc, par, gy, h=1e-6):
    """dL/dP by central differences of L = <gy, y_oracle(P)>."""
    g = np.zeros_like(sc.src.p)
    for k in range(sc.src.p.shape[0]):
        for a in range(3):
            sp, sm = sc.copy(), sc.copy()
            sp.src.p[k, a] += h
            sm.src.p[k, a] -= h
            g[k, a] = (np.sum(O.forward(sp, par) * gy) - np.sum(O.forward(sm, par) * gy)) / (2 * h)
    return g


CASES = [
    dict(seed=41, max_order=3, seconds=0.1, taps=32),
    dict(seed=42, max_order=4, seconds=0.12, taps=64, n_mics=2, moving_rcv=True),
    dict(seed=43, max_order=5, seconds=0.12, taps=96, n_knots=4, tiers=((2, 1), (4, 16), (99, 160))),
    # odd decimations: the gain/delay kernel keeps one output per lane, and the
    # gather's neighbouring outputs fall on two segments in most lanes
    dict(seed=49, max_order=3, seconds=0.1, taps=64, tiers=((1, 1), (2, 5), (99, 15))),
    # every image at the audio rate: one track segment per output
    dict(seed=50, max_order=2, seconds=0.06, taps=32, tiers=()),
]


@pytest.mark.parametrize("case", CASES)
def test_gradients_match_oracle(torch_cuda, case):
    sc, par = G.small_scene(**case)
    print("farrow backward case", case, flush=True)
    gy = np.random.default_rng(case["seed"]).standard_normal((sc.n_mics, sc.n_out))
    _, gx, gb, gs = gpu_backward([sc], farrow(par), [gy], torch_cuda)
    assert rel(gx, O.adjoint_x(sc, par, gy)) <= 1e-5
    assert rel(gb[0], O.grad_beta(sc, par, gy)) <= 1e-4
    ref = fd_knots(sc, par, gy)
    assert rel(gs, ref) <= 1e-3, (gs, ref)


def test_multi_scene_and_circle(torch_cuda):
    a, par = G.small_scene(seed=45, max_order=2, seconds=0.08, taps=64)
    b, _ = G.small_scene(seed=46, max_order=3, seconds=0.06, taps=64, circle=True)
    c, _ = G.small_scene(seed=47, max_order=2, seconds=0.05, taps=64, n_knots=2)
    rng = np.random.default_rng(6)
    gys = [rng.standard_normal((s.n_mics, s.n_out)) for s in (a, b, c)]
    plan, gx, gb, gs = gpu_backward([a, b, c], farrow(par), gys, torch_cuda)
    for s, (sc, gy) in enumerate(zip((a, b, c), gys)):
        o = plan.x_off[s]
        assert rel(gx[o:o + sc.n_in], O.adjoint_x(sc, par, gy)) <= 1e-5
        assert rel(gb[s], O.grad_beta(sc, par, gy)) <= 1e-4
    ka = a.src.p.shape[0]
    assert rel(gs[:ka], fd_knots(a, par, gys[0])) <= 1e-3
    assert rel(gs[ka:], fd_knots(c, par, gys[2])) <= 1e-3


def test_dot_product_identity_config2(torch_cuda):
    # <F x, gy> = <x, F^T gy> for the Farrow operator itself, at paper scale
    torch = torch_cuda
    scenes, par = G.config2()
    from paper_2508_03065_amd.msim import Plan
    plan = Plan(scenes, farrow(par))
    x = plan.pack_x([s.x for s in scenes])
    y = plan.forward(x)
    gy = torch.randn(plan.y_total, generator=torch.Generator().manual_seed(7)).cuda()
    gx, _, _ = plan.backward(x, gy, want_beta=False, want_src=False)
    assert plan.device_status() == 0
    lhs = torch.dot(y.double(), gy.double()).item()
    rhs = torch.dot(x.double(), gx.double()).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_config2_room_gradients(torch_cuda):
    # the paper-scale room and image count (K = 12, tiers) on a 0.25 s excerpt
    torch = torch_cuda
    scenes, par = G.config2(seconds=0.25)
    sc = scenes[0]
    from paper_2508_03065_amd.msim import Plan
    plan = Plan(scenes, farrow(par))
    x = plan.pack_x([sc.x])
    gy = np.random.default_rng(8).standard_normal((sc.n_mics, sc.n_out))
    gx, gb, _ = plan.backward(x, torch.from_numpy(gy.reshape(-1).astype(np.float32)).cuda(), want_src=False)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert rel(gx.cpu().numpy(), O.adjoint_x(sc, par, gy)) <= 1e-5
    assert rel(gb.cpu().numpy()[0], O.grad_beta(sc, par, gy)) <= 1e-4


def test_table_and_farrow_gradients_agree(torch_cuda):
    sc, par = G.small_scene(seed=48, max_order=6, seconds=0.2, taps=64, n_mics=2)
    gy = np.random.default_rng(10).standard_normal((sc.n_mics, sc.n_out))
    _, gxt, gbt, gst = gpu_backward([sc], par, [gy], torch_cuda)
    _, gxf, gbf, gsf = gpu_backward([sc], farrow(par), [gy], torch_cuda)
    assert rel(gxf, gxt) <= 5e-6
    assert rel(gbf, gbt) <= 5e-5
    assert rel(gsf, gst) <= 5e-4


def test_backward_deterministic(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    sc, par = G.small_scene(seed=49, max_order=5, seconds=0.15, taps=64, n_mics=2, moving_rcv=True)
    plan = Plan([sc], farrow(par))
    x = plan.pack_x([sc.x])
    gy = torch.randn(plan.y_total, generator=torch.Generator().manual_seed(11)).cuda()
    a = [t.clone() for t in plan.backward(x, gy)]
    b = [t.clone() for t in plan.backward(x, gy)]
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_autograd_function(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.autograd import scene_params, synthesize
    sc, par = G.small_scene(seed=50, max_order=3, seconds=0.08, taps=32)
    fpar = farrow(par)
    beta, knots = scene_params([sc])
    beta.requires_grad_(True)
    knots.requires_grad_(True)
    x = torch.from_numpy(sc.x).cuda().requires_grad_(True)
    target = torch.from_numpy(np.random.default_rng(12).standard_normal(sc.n_out) * 0.01).float().cuda()
    y = synthesize([sc], fpar, x, beta, knots)
    loss = 0.5 * ((y - target) ** 2).sum()
    loss.backward()
    gy = (y.detach() - target).double().cpu().numpy().reshape(1, -1)
    assert rel(x.grad.cpu().numpy(), O.adjoint_x(sc, par, gy)) <= 1e-5
    assert rel(beta.grad[0].numpy(), O.grad_beta(sc, par, gy)) <= 1e-4
    assert rel(knots.grad.numpy(), fd_knots(sc, par, gy)) <= 1e-3
