"""torch.autograd binding of the synthesis: gradients with respect to the
source signal, the six wall coefficients of every scene and the knot positions
of piecewise-linear source paths.  Both directions run in libmsim.so (the
batched forward and backward, replayed from HIP graphs); this module keeps one
plan per set of scenes, rewrites its coefficients and knots in place before a
call (msim_plan_update), and moves tensors across the boundary."""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import scenegen as G
from ._lib import MsimError
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


class Synthesizer:
    """One plan over a fixed set of scenes whose wall coefficients and source knots
    change between calls (a training loop): the plan's delay bounds are widened by
    `knot_slack` metres, updates within it are written in place, and a knot that
    moves further makes a new plan around the current path."""

    def __init__(self, scenes: Sequence, par, knot_slack: float = 0.05):
        self.scenes = list(scenes)
        self.par = dataclasses.replace(par, knot_slack=float(knot_slack))
        self.plan: Optional[Plan] = None
        self.replans = 0
        self._beta = self._knots = None
        self._y = self._out = None

    def prepare(self, beta: np.ndarray, knots: np.ndarray) -> Plan:
        if self.plan is None:
            self.plan = Plan(_with_params(self.scenes, beta, knots), self.par)
        elif not (np.array_equal(beta, self._beta) and np.array_equal(knots, self._knots)):
            try:
                self.plan.update(beta, knots)
            except MsimError:
                # beyond the slack: plan around the current path
                self.plan = Plan(_with_params(self.scenes, beta, knots), self.par)
                self._y = self._out = None
                self.replans += 1
        self._beta, self._knots = beta.copy(), knots.copy()
        return self.plan

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        plan = self.plan
        if self._y is None:
            self._y = torch.empty(plan.y_total, dtype=torch.float32, device=x.device)
        plan.forward_batched(x, self._y)
        return self._y.clone()

    def backward(self, x: torch.Tensor, gy: torch.Tensor, nx: bool, nb: bool, nk: bool):
        plan = self.plan
        if self._out is None or (self._out[0] is None) != (not nx) or (self._out[1] is None) != (not nb) \
                or (self._out[2] is None) != (not nk):
            plan.backward(x, gy, want_x=nx, want_beta=nb, want_src=nk, batched=True)
            self._out = plan.last_backward_buffers
        else:
            plan.backward(x, gy, want_x=nx, want_beta=nb, want_src=nk, batched=True, out=self._out)
        gx, gb, gs = self._out
        return (gx.clone() if gx is not None else None, gb.clone() if gb is not None else None,
                gs[: plan.src_total].clone() if gs is not None else None)

    def __call__(self, x: torch.Tensor, beta: torch.Tensor, knots: torch.Tensor) -> torch.Tensor:
        return MovingISMFn.apply(x, beta, knots, self)


class MovingISMFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, beta, knots, synth: Synthesizer):
        b = beta.detach().cpu().numpy().astype(np.float64)
        kn = knots.detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
        synth.prepare(b, kn)
        xx = x.detach().contiguous()
        y = synth.forward(xx)
        ctx.synth = synth
        ctx.params = (b, kn)
        ctx.beta_dev, ctx.knots_dev = beta.device, knots.device
        ctx.save_for_backward(xx)
        return y

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        nx, nb, nk = ctx.needs_input_grad[:3]
        synth = ctx.synth
        synth.prepare(*ctx.params)     # the parameters of this forward, should another call have changed them
        gx, gb, gs = synth.backward(x, gy.detach().contiguous().float(), nx, nb, nk)
        gb = gb.to(ctx.beta_dev) if gb is not None else None
        gs = gs.to(ctx.knots_dev) if gs is not None else None
        return gx, gb, gs, None


def synthesize(scenes: Sequence, par, x: torch.Tensor, beta: torch.Tensor, knots: torch.Tensor,
               synth: Optional[Synthesizer] = None) -> torch.Tensor:
    """Differentiable y (packed, [y_total]) for packed source signals x; pass the
    same `synth` (a Synthesizer over these scenes) across calls to keep its plan."""
    if synth is None:
        synth = Synthesizer(scenes, par)
    return synth(x, beta, knots)
