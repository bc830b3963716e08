"""torch.autograd binding of the synthesis: gradients with respect to the
source signal, the six wall coefficients of every scene and the knot positions
of piecewise-linear source paths.  Both directions run in libmsim.so
(msim_forward / msim_backward); this module only rebuilds the plan from the
current coefficient and knot values and moves tensors across the boundary."""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import torch

from . import scenegen as G
from .msim import Plan


def scene_params(scenes: Sequence) -> Tuple[torch.Tensor, torch.Tensor]:
    """(beta [S, 6], knots [sum of PWL source knots, 3]) of the scenes, FP64."""
    beta = torch.tensor(np.stack([np.asarray(s.beta, np.float64) for s in scenes]))
    kn = [np.asarray(s.src.p, np.float64).reshape(-1, 3) for s in scenes if s.src.kind == G.PWL]
    knots = torch.tensor(np.concatenate(kn) if kn else np.zeros((0, 3)))
    return beta, knots


def _with_params(scenes: Sequence, beta: np.ndarray, knots: np.ndarray) -> List:
    out, k = [], 0
    for s, sc in enumerate(scenes):
        c = sc.copy()
        c.beta = beta[s].copy()
        if c.src.kind == G.PWL:
            n = c.src.p.shape[0]
            c.src.p = knots[k:k + n].copy()
            k += n
        out.append(c)
    return out


class MovingISMFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, beta, knots, scenes, par):
        b = beta.detach().cpu().numpy().astype(np.float64)
        kn = knots.detach().cpu().numpy().astype(np.float64)
        plan = Plan(_with_params(scenes, b, kn), par)
        xx = x.detach().contiguous()
        y = plan.forward(xx)
        ctx.plan = plan
        ctx.beta_dev, ctx.knots_dev = beta.device, knots.device
        ctx.save_for_backward(xx)
        return y

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        nx, nb, nk = ctx.needs_input_grad[:3]
        gx, gb, gs = ctx.plan.backward(x, gy.detach().contiguous().float(), want_x=nx, want_beta=nb, want_src=nk)
        gb = gb.to(ctx.beta_dev) if gb is not None else None
        gs = gs.to(ctx.knots_dev) if gs is not None else None
        return gx, gb, gs, None, None


def synthesize(scenes: Sequence, par, x: torch.Tensor, beta: torch.Tensor, knots: torch.Tensor) -> torch.Tensor:
    """Differentiable y (packed, [y_total]) for packed source signals x."""
    return MovingISMFn.apply(x, beta, knots, list(scenes), par)
