"""In-place parameter updates (msim_plan_update) and the autograd binding that
keeps one plan across calls: after new wall coefficients and knot positions
the plan's output and gradients match the oracle at the new parameters, a knot
moved beyond the planned slack is refused (and the Synthesizer plans again),
and a refused update changes nothing."""
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


def two_scenes():
    a, par = G.small_scene(seed=61, max_order=3, seconds=0.08, taps=64, n_knots=3)
    b, _ = G.small_scene(seed=62, max_order=4, seconds=0.06, taps=64, n_knots=4, n_mics=2)
    return [a, b], par


@pytest.mark.parametrize("fd", [0, 1], ids=["table", "farrow"])
def test_update_matches_oracle(torch_cuda, fd):
    torch = torch_cuda
    from paper_2508_03065_amd.msim import Plan
    from paper_2508_03065_amd._lib import MsimError
    scenes, par = two_scenes()
    par = dataclasses.replace(par, fd_kind=fd, knot_slack=0.05)
    plan = Plan(scenes, par)
    x = plan.pack_x([s.x for s in scenes])
    y0 = plan.forward_batched(x).clone()
    rng = np.random.default_rng(3)
    new = [s.copy() for s in scenes]
    for s in new:
        s.beta = np.clip(s.beta + rng.uniform(-0.05, 0.05, 6), 0.0, 1.0)
        s.src.p = s.src.p + rng.uniform(-0.03, 0.03, s.src.p.shape)
    plan.update(np.stack([s.beta for s in new]), np.concatenate([s.src.p for s in new]))
    y = plan.forward_batched(x)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    for s, yv in zip(new, plan.unpack_y(y)):
        assert rel(yv.cpu().numpy(), O.forward(s, par)) <= 1e-5
    gy = [np.random.default_rng(9 + k).standard_normal((s.n_mics, s.n_out)) for k, s in enumerate(new)]
    gyt = torch.from_numpy(np.concatenate([g.reshape(-1) for g in gy]).astype(np.float32)).cuda()
    gx, gb, gs = plan.backward(x, gyt, batched=True)
    torch.cuda.synchronize()
    for k, s in enumerate(new):
        o = plan.x_off[k]
        assert rel(gx[o:o + s.n_in].cpu().numpy(), O.adjoint_x(s, par, gy[k])) <= 1e-5
        assert rel(gb[k].cpu().numpy(), O.grad_beta(s, par, gy[k])) <= 1e-4
    # beyond the slack, or a coefficient above 1: refused, and the plan unchanged
    far = np.concatenate([s.src.p for s in new]) + 0.2
    with pytest.raises(MsimError, match="knot_slack"):
        plan.update(None, far)
    bad = np.stack([s.beta for s in new])
    bad[0, 0] = 1.5
    with pytest.raises(MsimError):
        plan.update(bad, None)
    assert torch.equal(plan.forward_batched(x), y)
    # and back to the original parameters: the original output, bit for bit
    plan.update(np.stack([s.beta for s in scenes]), np.concatenate([s.src.p for s in scenes]))
    assert torch.equal(plan.forward_batched(x), y0)


def test_synthesizer_training_steps(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd.autograd import Synthesizer, scene_params
    scenes, par = two_scenes()
    synth = Synthesizer(scenes, par, knot_slack=0.05)
    beta, knots = scene_params(scenes)
    x = synth_x = None
    target = None
    for step in range(3):
        beta_p = beta.clone().requires_grad_(True)
        knots_p = knots.clone().requires_grad_(True)
        if x is None:
            from paper_2508_03065_amd.msim import Plan
            x = Plan(scenes, par).pack_x([s.x for s in scenes]).requires_grad_(True)
            g = np.random.default_rng(5).standard_normal(sum(s.n_mics * s.n_out for s in scenes)) * 0.01
            target = torch.from_numpy(g).float().cuda()
        y = synth(x, beta_p, knots_p)
        loss = 0.5 * ((y - target) ** 2).sum()
        loss.backward()
        # the oracle at this step's parameters
        cur = []
        k = 0
        for s in scenes:
            c = s.copy()
            c.beta = beta[len(cur)].numpy().copy()
            n = c.src.p.shape[0]
            c.src.p = knots[k:k + n].numpy().copy()
            k += n
            cur.append(c)
        gyv = (y.detach() - target).double().cpu().numpy()
        off = 0
        for i, c in enumerate(cur):
            gy = gyv[off:off + c.n_mics * c.n_out].reshape(c.n_mics, c.n_out)
            off += c.n_mics * c.n_out
            assert rel(beta_p.grad[i].numpy(), O.grad_beta(c, par, gy)) <= 1e-4
        # a small gradient step, then at step 2 a knot jump beyond the slack
        with torch.no_grad():
            beta = torch.clamp(beta - 0.01 * torch.sign(beta_p.grad), 0.0, 1.0)
            knots = knots - 0.01 * torch.sign(knots_p.grad)
            if step == 1:
                knots[0, 0] += 0.1
    assert synth.replans == 1
