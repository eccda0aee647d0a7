"""Differentiable rollouts: gradients of a loss of the final macroscopic
fields with respect to the initial velocity field and beta.

``rollout(ux0, uy0, beta, nsteps, ...)`` returns (rho, u_x, u_y) at
t = nsteps; all of its arithmetic runs in libkbc.  The forward pass keeps the
population state every K steps (K = ceil(sqrt(nsteps)) by default); the
backward pass walks the segments from last to first, recomputes the K states
of a segment from its checkpoint into K - 1 slots, and runs the hand-written
adjoint step kernel back through them, then the adjoint of the initial state.
By default (``overlap=True``) one native call runs all segments: each launch
runs one adjoint step of the current segment and one recomputation step of
the next, which uses a second slot set.  Memory is about 2 sqrt(nsteps) states (3 with overlap); the
recomputation adds one forward step per step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .sim import Sim


@dataclass
class RolloutConfig:
    nsteps: int
    collision: str = "kbc"
    variant: str = "B"
    form: str = "f32"
    init: str = "grad_cd"
    checkpoint_every: int | None = None
    gamma_mode: str = "estimate"
    gamma_guard: float = 1e-12
    tile: tuple | None = None
    gamma_grad: str = "full"      # "full": differentiate gamma(f); "frozen": hold it
    overlap: bool = True          # recompute the next segment inside the adjoint launches (two slot sets)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ux0, uy0, beta, cfg: RolloutConfig):
        ny, nx = ux0.shape
        dev = ux0.device
        sim = Sim(nx, ny, float(beta), collision=cfg.collision, variant=cfg.variant, form=cfg.form,
                  gamma_mode=cfg.gamma_mode, gamma_guard=cfg.gamma_guard, device=dev, tile=cfg.tile)
        ux0d = ux0.detach().to(torch.float64).contiguous()
        uy0d = uy0.detach().to(torch.float64).contiguous()
        sim.init(ux0d, uy0d, mode=cfg.init)
        sim.set_adjoint_gamma(cfg.gamma_grad == "frozen")
        N = int(cfg.nsteps)
        K = cfg.checkpoint_every or max(1, math.ceil(math.sqrt(max(N, 1))))
        ckpts = {}
        for s in range(0, N, K):
            ckpts[s] = sim.state_buffer().clone()
            sim.step(min(K, N - s))
        rho, ux, uy = sim.moments()
        ctx.sim, ctx.ckpts, ctx.K, ctx.N, ctx.cfg = sim, ckpts, K, N, cfg
        ctx.final = sim.state_buffer()
        ctx.save_for_backward(ux0d, uy0d)
        ctx.beta_shape = beta.shape if isinstance(beta, torch.Tensor) else None
        return rho, ux, uy

    @staticmethod
    def backward(ctx, grho, gux, guy):
        sim: Sim = ctx.sim
        ux0, uy0 = ctx.saved_tensors
        K, N = ctx.K, ctx.N
        dev = ux0.device
        lam_a, lam_b = sim.new_adjoint(), sim.new_adjoint()
        acc = torch.zeros(1, dtype=torch.float64, device=dev)
        sim.adjoint_seed(ctx.final, lam_a, grho, gux, guy)
        nslot = max(0, min(K, N) - 1)
        slots = [sim.new_state() for _ in range(nslot)]
        if ctx.cfg.overlap and len(ctx.ckpts) > 1:
            slots_b = [sim.new_state() for _ in range(nslot)]
            ckpts = [ctx.ckpts[s] for s in sorted(ctx.ckpts.keys())]
            if sim.adjoint_rollout(ckpts, N, K, slots, slots_b, lam_a, lam_b, acc):
                lam_a, lam_b = lam_b, lam_a
        else:
            for s in sorted(ctx.ckpts.keys(), reverse=True):
                k = min(s + K, N) - s
                if sim.adjoint_segment(ctx.ckpts[s], slots, k, lam_a, lam_b, acc):
                    lam_a, lam_b = lam_b, lam_a
        gx = torch.empty_like(ux0)
        gy = torch.empty_like(uy0)
        sim.adjoint_init(ux0, uy0, lam_a, gx, gy, acc, mode=ctx.cfg.init)
        gbeta = None
        if ctx.beta_shape is not None:
            gbeta = acc.reshape(ctx.beta_shape)
        ctx.sim = None
        ctx.ckpts = None
        return gx, gy, gbeta, None


def rollout(ux0: torch.Tensor, uy0: torch.Tensor, beta, nsteps: int, **kw):
    """(rho, u_x, u_y) after `nsteps` steps from the initial velocity (ux0, uy0)
    ([ny, nx] float64 tensors on the GPU) and beta (float or 0-d tensor);
    differentiable in ux0, uy0 and beta.  Keyword arguments: see RolloutConfig."""
    cfg = RolloutConfig(nsteps=nsteps, **kw)
    if not isinstance(beta, torch.Tensor):
        beta = torch.tensor(float(beta), dtype=torch.float64, device=ux0.device)
    return _Rollout.apply(ux0, uy0, beta, cfg)
