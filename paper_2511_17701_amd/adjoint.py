"""Differentiable frozen-field particle push (the differentiation form).

`FrozenFieldPush.apply(u0, B0, run)` advances particles `run.steps` push
steps (grpic_push) in the frozen initial field of amplitude B0 (the Wald
field, or the monopole field of the BZ test, built by the library's
grpic_fields_init_* call for that B0) and returns their final state
(x1, x2, u1, u2, u3) as an (n, 5) float64 tensor, x = cell + offset.  Its
backward is the adjoint sweep: the forward pass keeps the particle state
every `run.every` steps (checkpoints); the backward pass replays each segment
from its checkpoint, keeping the state of every step, and calls
grpic_push_adjoint once per step in reverse order.  It returns the gradient
with respect to the initial momenta u0 (n, 3) and the amplitude B0.

All arithmetic runs in libgrpic (grpic_push, grpic_push_adjoint); this module
only sequences the calls and moves tensors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import grpic

STATE_KEYS = ("i1", "i2", "dx1", "dx2", "u1", "u2", "u3", "w", "phi", "i1p", "i2p", "dx1p",
              "dx2p", "tag")


@dataclass
class FrozenRun:
    """What the differentiable push needs besides (u0, B0)."""
    ctx: "grpic.Context"       # FP64 context; n_iter large enough for the fixed points
    start: dict                # particle arrays; u1..u3 are replaced by u0
    steps: int
    every: int = 10
    init: str = "wald"         # initial field: "wald" or "monopole" (linear in B0)
    stats: dict = field(default_factory=dict)

    def fields(self, b0: float) -> torch.Tensor:
        """The frozen field set of amplitude b0, built by libgrpic."""
        F = self.ctx.new_fields(self.start["u1"].device)
        if self.init == "wald":
            self.ctx.fields_init_wald(F, b0)
        elif self.init == "monopole":
            self.ctx.fields_init_monopole(F, b0)
        else:
            raise ValueError(f"unknown initial field {self.init!r}")
        return F


def _copy(P):
    return {k: v.clone() for k, v in P.items()}


def final_state(P):
    return torch.stack([P["i1"].double() + P["dx1"], P["i2"].double() + P["dx2"],
                        P["u1"], P["u2"], P["u3"]], dim=1)


class FrozenFieldPush(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, B0, run: FrozenRun):
        if u0.dtype != torch.float64 or u0.dim() != 2 or u0.shape[1] != 3:
            raise ValueError("u0 must be an (n, 3) float64 tensor")
        b0 = float(B0)
        F = run.fields(b0)
        P = _copy(run.start)
        P["u1"], P["u2"], P["u3"] = (u0[:, c].contiguous().clone() for c in range(3))
        checkpoints = []
        for s in range(run.steps):
            if s % run.every == 0:
                checkpoints.append(_copy(P))
            run.ctx.push(F, P)
        ctx.run, ctx.F, ctx.b0, ctx.checkpoints = run, F, b0, checkpoints
        ctx.b0_device = B0.device if torch.is_tensor(B0) else torch.device("cpu")
        return final_state(P)

    @staticmethod
    def backward(ctx, gout):
        run, F, b0 = ctx.run, ctx.F, ctx.b0
        n = gout.shape[0]
        g = gout.t().contiguous().clone()          # rows x1, x2, u1, u2, u3
        gB0 = torch.zeros(n, dtype=torch.float64, device=gout.device)
        for seg in reversed(range(len(ctx.checkpoints))):
            P = _copy(ctx.checkpoints[seg])
            count = min(run.every, run.steps - seg * run.every)
            states = []
            for _ in range(count):
                states.append(_copy(P))
                run.ctx.push(F, P)
            for S in reversed(states):
                run.ctx.push_adjoint(F, b0, S, g, g, gB0)
        run.stats["gB0_per_particle"] = gB0
        grad_u0 = g[2:5].t().contiguous() if ctx.needs_input_grad[0] else None
        grad_B0 = gB0.sum().reshape(()).to(ctx.b0_device) if ctx.needs_input_grad[1] else None
        return grad_u0, grad_B0, None
