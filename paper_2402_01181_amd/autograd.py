"""Differentiable rollouts: a torch.autograd.Function whose backward is the
library's hand-written adjoint (checkpointed, recomputed in reverse).

    x, v = MPMRollout.apply(E, nu, u, sim, n_substeps)

E, nu: [n_envs] tensors (Young's modulus, Poisson's ratio, Sec. III-B Lame
relation); u: [n_envs][max_tools][n_substeps][3] per-substep tool
velocities.  The rollout restarts from the Sim's initial state every call.
Outputs are the final positions and velocities, (Ntot, 3), original order.
"""
from __future__ import annotations

import torch


class MPMRollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, E, nu, u, sim, n_substeps):
        n = int(n_substeps)
        if sim.max_tape < n:
            raise ValueError(f"the Sim was created with max_tape={sim.max_tape} < {n}")
        with torch.no_grad():
            sim.material[:, 0] = E.detach().to(sim.material)
            sim.material[:, 1] = nu.detach().to(sim.material)
            for (e, t), traj in sim.traj.items():
                traj[:n] = u[e, t].detach().to(traj)
            sim.reset()
            sim.step(n, record_tape=True)
            x = sim.positions()
            v = sim.velocities()
        ctx.sim, ctx.n = sim, n
        ctx.like = tuple((t.device, t.dtype) for t in (E, nu, u))
        return x, v

    @staticmethod
    def backward(ctx, gx, gv):
        sim, n = ctx.sim, ctx.n
        xbar = None if gx is None else gx.detach().to(torch.float32).T.contiguous()
        vbar = None if gv is None else gv.detach().to(torch.float32).T.contiguous()
        g = sim.adjoint(n, xbar=xbar, vbar=vbar)
        (dE, tE), (dnu, tnu), (du, tu) = ctx.like
        return g["gE"].to(dE, tE), g["gnu"].to(dnu, tnu), g["gu"].to(du, tu), None, None
