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
        ctx.dtypes = (E.dtype, nu.dtype, u.dtype)
        return x, v

    @staticmethod
    def backward(ctx, gx, gv):
        sim, n = ctx.sim, ctx.n
        xbar = None if gx is None else gx.detach().to(torch.float32).T.contiguous()
        vbar = None if gv is None else gv.detach().to(torch.float32).T.contiguous()
        g = sim.adjoint(n, xbar=xbar, vbar=vbar)
        dE, dnu, du = ctx.dtypes
        return g["gE"].to(dE), g["gnu"].to(dnu), g["gu"].to(du), None, None
