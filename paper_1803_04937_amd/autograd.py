"""Differentiable rollout: J(f_T) of a lattice started from f_0 = f^eq(1, u_init),
with gradients with respect to u_init, the body acceleration a and omega.

Forward: lbm_init, then T fused stream-collide steps, storing the state every
C steps (checkpoints); J and its seed lam_T = dJ/df_T come from
lbm_objective.  Backward: for each segment from last to first, the states of
the segment are recomputed from its checkpoint into a ring of C buffers with
lbm_stream_collide, then lbm_adjoint_step runs backwards through them
(lam_t = (d f_{t+1} / d f_t)^T lam_{t+1}, parameter gradients accumulated in
FP64 on the device); finally lbm_init_vjp maps lam_0 to dJ/du_init.  Memory:
ceil(T / C) checkpoints + C ring buffers + 2 adjoint fields; C defaults to
ceil(sqrt(T)).

For the 16-bit storage formats the adjoint linearises at the dequantised
stored states and treats the quantisation as the identity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import capi
from .lattice import Lattice


@dataclass
class RolloutConfig:
    nx: int
    ny: int
    nz: int
    steps: int
    periodic: tuple = (1, 1, 1)
    equilibrium: str = "improved"
    collision: str = "srt"
    dtype: str = "f32"
    trt_magic: float = 3.0 / 16.0
    objective: int = capi.LBM_OBJ_KINETIC_ENERGY
    checkpoint_every: int | None = None
    solid: torch.Tensor | None = field(default=None, repr=False)
    scale: float = 0.0
    rounding: str = "nearest"
    seed: int = 0
    stencil: int = 19
    mrt_omega3: float = 1.0
    mrt_omega4: float = 1.0
    # lambda at solid cells is never read here (the objective seeds zero
    # there, the initial-state VJP ignores it), so the adjoint skips it
    adjoint_solid: str = "skip"

    @property
    def segment(self) -> int:
        if self.checkpoint_every:
            return int(self.checkpoint_every)
        return max(1, math.ceil(math.sqrt(self.steps)))


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_init, accel, omega, cfg: RolloutConfig):
        u_init = u_init.detach().to(torch.float64).contiguous()
        lat = Lattice(cfg.nx, cfg.ny, cfg.nz, u=u_init, solid=cfg.solid, periodic=cfg.periodic,
                      equilibrium=cfg.equilibrium, collision=cfg.collision, dtype=cfg.dtype,
                      omega=float(omega), trt_magic=cfg.trt_magic,
                      accel=tuple(float(v) for v in accel.detach().cpu()), scale=cfg.scale,
                      rounding=cfg.rounding, seed=cfg.seed, stencil=cfg.stencil,
                      mrt_omega3=cfg.mrt_omega3, mrt_omega4=cfg.mrt_omega4,
                      adjoint_solid=cfg.adjoint_solid, device=u_init.device)
        C = cfg.segment
        ckpts = {}
        for t in range(cfg.steps):
            if t % C == 0:
                ckpts[t] = lat.new_state()
                lat.copy_state(lat.state, ckpts[t])
            lat.step(1)
        out = torch.zeros(4, dtype=torch.float64, device=u_init.device)
        lam_T = lat.new_adjoint(zero=False)
        lat.objective(cfg.objective, lat.state, out, lam_T)
        ctx.lat, ctx.cfg, ctx.ckpts, ctx.lam_T, ctx.out = lat, cfg, ckpts, lam_T, out
        ctx.param_devices = (accel.device, accel.dtype, omega.device, omega.dtype)
        ctx.save_for_backward(u_init)
        return out[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        (u_init,) = ctx.saved_tensors
        lat, cfg = ctx.lat, ctx.cfg
        T, C = cfg.steps, cfg.segment
        grad = torch.zeros(4, dtype=torch.float64, device=u_init.device)
        grad[1:] += ctx.out[1:]                 # explicit dJ/da of the objective
        lam_next = ctx.lam_T
        lam_prev = lat.new_adjoint(zero=False)
        ring = [None] + [lat.new_state() for _ in range(min(C, T) - 1)]
        for start in reversed(range(0, T, C)):
            end = min(start + C, T)
            ring[0] = ctx.ckpts[start]
            for k in range(1, end - start):
                lat.stream_collide(ring[k - 1], ring[k], start + k - 1)
            for t in reversed(range(start, end)):
                lat.adjoint_step(ring[t - start], lam_next, lam_prev, grad)
                lam_next, lam_prev = lam_prev, lam_next
        grad_u = torch.empty_like(u_init)
        lat.init_vjp(u_init, lam_next, grad_u)
        ctx.lat = ctx.ckpts = ctx.lam_T = None
        lat.close()
        g = gJ.to(device=u_init.device, dtype=torch.float64)
        adev, adt, wdev, wdt = ctx.param_devices
        return (g * grad_u, (g * grad[1:4]).to(adev, adt), (g * grad[0]).to(wdev, wdt), None)


def rollout_objective(u_init: torch.Tensor, accel: torch.Tensor, omega: torch.Tensor,
                      cfg: RolloutConfig) -> torch.Tensor:
    """J(f_T) as a differentiable function of u_init (3, nz, ny, nx), accel (3,)
    and omega (scalar tensor)."""
    return _Rollout.apply(u_init, accel, omega, cfg)
