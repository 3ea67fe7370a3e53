"""Differentiable rollout of the T2S2-FDLBM step with sqrt(N) checkpointing.

``T2S2Rollout.apply(rho0, ux0, uy0, nu, spec)`` starts from the equilibrium
state f~ = f^eq(rho0, u0), takes ``spec.nsteps`` steps on the GPU through the
C-ABI, and returns the final velocity (ux, uy).  Its backward pass runs the
hand-written discrete adjoint of every step in reverse: the state is stored
every K = ceil(sqrt(N)) steps during the forward pass, and each segment is
recomputed from its checkpoint before its adjoint steps run (memory about
sqrt(N) checkpoints plus one segment's states and S instead of N states).
Gradients: dL/drho0, dL/dux0, dL/duy0 (whole fields) and dL/dnu at a fixed
dt, which the adjoint steps accumulate on the device.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Any, Optional

import torch

from . import Context, make_config


@dataclasses.dataclass
class RolloutSpec:
    """Mesh and scheme of a rollout (everything but the differentiated inputs)."""

    x: Any
    y: Any
    periodic_x: bool
    periodic_y: bool
    period_x: float = 0.0
    period_y: float = 0.0
    cfl: float = 0.0
    dt: float = 0.0
    eta: float = 0.1
    A: float = 0.5
    u_wall: Any = None
    storage: str = "f64"
    nsteps: int = 1
    checkpoint_every: Optional[int] = None
    device: Any = None
    # Backward pass: True keeps each step's new state and S while it walks a
    # segment back (t2s2_step_save_s / t2s2_adjoint_step_stored: one forward
    # step per time step instead of two); False recomputes the step inside
    # each adjoint step (memory: two state copies); None chooses True when a
    # segment's states and S take under a quarter of the free device memory.
    store_s: Optional[bool] = None

    def context(self, nu: float) -> Context:
        cfg = make_config(nu=nu, cfl=self.cfl, dt=self.dt, eta=self.eta, A=self.A,
                          u_wall=self.u_wall, periodic_x=self.periodic_x,
                          periodic_y=self.periodic_y, period_x=self.period_x,
                          period_y=self.period_y, storage=self.storage)
        return Context(cfg, self.x, self.y, device=self.device)

    def segment(self) -> int:
        if self.checkpoint_every:
            return max(1, int(self.checkpoint_every))
        return max(1, math.ceil(math.sqrt(self.nsteps)))


def forward_velocity(spec: RolloutSpec, rho0, ux0, uy0, nu: float):
    """Plain forward run (no checkpoints): final (ux, uy)."""
    sim = spec.context(nu)
    sim.init_macro(rho0, ux0, uy0)
    sim.step(spec.nsteps)
    _, u, v = sim.moments()
    return u, v


class T2S2Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, ux0, uy0, nu, spec: RolloutSpec):
        nu_val = float(nu)
        sim = spec.context(nu_val)
        sim.init_macro(rho0, ux0, uy0)
        K = spec.segment()
        checkpoints = []
        done = 0
        while done < spec.nsteps:
            checkpoints.append((done, sim.save_state()))
            n = min(K, spec.nsteps - done)
            sim.step(n)
            done += n
        _, u, v = sim.moments()
        ctx.sim = sim
        ctx.spec = spec
        ctx.checkpoints = checkpoints
        ctx.final_state = sim.save_state()
        ctx.nu = nu_val
        ctx.save_for_backward(rho0, ux0, uy0)
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        rho0, ux0, uy0 = ctx.saved_tensors
        sim: Context = ctx.sim
        sim.enable_adjoint()
        lam_a, lam_b = sim.adjoint_buffer(), sim.adjoint_buffer()
        gu = gu if gu is not None else torch.zeros_like(ux0)
        gv = gv if gv is not None else torch.zeros_like(uy0)
        sim.adjoint_seed_velocity(ctx.final_state, gu, gv, lam_a)
        dnu = torch.zeros(1, dtype=torch.float64, device=sim.device)
        store_s = ctx.spec.store_s
        if store_s is None:
            seg = ctx.spec.segment() * (ctx.final_state.numel() + lam_a.numel())
            store_s = seg < torch.cuda.mem_get_info(sim.device)[0] // 4
        if store_s:
            # one segment's states after its checkpoint and its S, reused
            K = ctx.spec.segment()
            seg_states = [torch.empty_like(ctx.final_state) for _ in range(K)]
            seg_s = [sim.adjoint_buffer() for _ in range(K)]
        for start, saved in reversed(ctx.checkpoints):
            n = min(ctx.spec.segment(), ctx.spec.nsteps - start)
            if store_s:
                # states[k + 1] = step(states[k]), with its S in seg_s[k]
                states = [saved] + seg_states[:n]
                for k in range(n):
                    sim.step_save_s(states[k], states[k + 1], seg_s[k])
                for k in range(n - 1, -1, -1):
                    sim.adjoint_step_stored(states[k], states[k + 1], seg_s[k], lam_a, lam_b,
                                            dnu)
                    lam_a, lam_b = lam_b, lam_a
                continue
            sim.restore_state(saved)
            states = [sim.save_state()]
            for _ in range(n - 1):
                sim.step(1)
                states.append(sim.save_state())
            for k in range(n - 1, -1, -1):
                sim.adjoint_step(states[k], lam_a, lam_b, dnu)
                lam_a, lam_b = lam_b, lam_a
            del states
        if store_s:
            del seg_states, seg_s
        grho, gux, guy = sim.adjoint_init_macro(lam_a, rho0, ux0, uy0)
        return grho, gux, guy, dnu.reshape(()), None
