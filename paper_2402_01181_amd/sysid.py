"""Stiffness sweeps and material identification on top of the substep and its
hand adjoint.

The paper presses the same tissue with four Young's moduli and shows that
stiffer tissue deforms less (Sec. IV, Fig. seq2); it names differentiable
simulation as future work (Sec. V).  Two tools built on the library:

* ``stiffness_sweep``: one batched run with an environment per modulus;
  returns each environment's largest and mean particle displacement.
* ``identify``: recover (E, nu) of a tissue from an observed final particle
  configuration by L-BFGS through ``MPMRollout`` (gradients from
  ``mpm_substep_adjoint``), on log E and nu = (1 + tanh q) / 4, which keeps
  nu inside (0, 0.5).

Both run on the GPU only, like the rest of the package.
"""
from __future__ import annotations

import copy
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .scenes import Scene
from .sim import Sim


def stiffness_sweep(scene: Scene, E_values: Sequence[float], substeps: int,
                    options: Optional[Dict[int, int]] = None) -> Dict[str, np.ndarray]:
    """Largest and mean particle displacement after ``substeps`` for each
    modulus in ``E_values`` ({"max": [len(E_values)], "mean": [...]});
    environment 0 of ``scene`` is copied once per value and all copies run
    in one batched call."""
    base = scene.envs[0]
    envs = []
    for E in E_values:
        e = copy.deepcopy(base)
        e.E = float(np.float32(E))
        envs.append(e)
    sc = Scene(f"{scene.name}-sweep", envs, dt=scene.dt, substeps=substeps, gravity=scene.gravity,
               bound=scene.bound)
    sim = Sim(sc, options=options)
    try:
        sim.step(substeps)
        dmax, dmean = [], []
        for k, e in enumerate(envs):
            x = sim.read(L.F_X, k, device=False).T.astype(np.float64)
            d = np.linalg.norm(x - e.x.astype(np.float64), axis=1)
            dmax.append(float(d.max()))
            dmean.append(float(d.mean()))
        if any(sim.read(L.F_STATUS, k) for k in range(len(envs))):
            raise RuntimeError("a sweep environment raised a status flag")
        return {"max": np.array(dmax), "mean": np.array(dmean)}
    finally:
        sim.close()


def identify(scene: Scene, x_obs: torch.Tensor, E0: float, nu0: float, substeps: int,
             max_evals: int = 40, checkpoint_every: int = 20,
             options: Optional[Dict[int, int]] = None) -> Dict[str, object]:
    """Fit (E, nu) of environment 0 so that its particle positions after
    ``substeps`` match ``x_obs`` ((N, 3), original particle order), with the
    scene's tool trajectories held fixed.  Loss: mean squared distance,
    divided by the mean squared displacement of ``x_obs`` from the start.
    Returns the fitted values and the history of evaluations."""
    scene = copy.deepcopy(scene)
    env = scene.envs[0]
    for tool in env.tools:          # one velocity per substep, the last one held as the library does
        tr = np.asarray(tool.traj, np.float32)
        tool.traj = tr[np.minimum(np.arange(substeps), tr.shape[0] - 1)]
    sim = Sim(scene, max_tape=substeps, checkpoint_every=checkpoint_every, options=options)
    from .autograd import MPMRollout
    dev = sim.device
    x_obs = x_obs.to(dev, torch.float64)
    x0 = torch.as_tensor(env.x, dtype=torch.float64, device=dev)
    scale = float(((x_obs - x0) ** 2).sum(1).mean())
    if not scale > 0:
        raise ValueError("the observed configuration equals the initial one")
    # fixed tool trajectories: [n_envs][max_tools][substeps][3]
    u = torch.zeros((1, sim.max_tools, substeps, 3), dtype=torch.float64)
    for t, tool in enumerate(env.tools):
        u[0, t] = torch.from_numpy(np.asarray(tool.traj, np.float64))
    logE = torch.tensor([np.log(E0)], dtype=torch.float64, requires_grad=True)
    q = torch.tensor([np.arctanh(4.0 * nu0 - 1.0)], dtype=torch.float64, requires_grad=True)
    history: List[dict] = []

    def params():
        return torch.exp(logE), 0.25 * (1.0 + torch.tanh(q))

    opt = torch.optim.LBFGS([logE, q], lr=1.0, max_iter=max_evals, max_eval=max_evals,
                            tolerance_grad=1e-12, tolerance_change=1e-14, history_size=10,
                            line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        E, nu = params()
        x, _ = MPMRollout.apply(E, nu, u, sim, substeps)
        loss = ((x.double() - x_obs) ** 2).sum(1).mean() / scale
        loss.backward()
        history.append({"E": float(E.detach()), "nu": float(nu.detach()), "loss": float(loss.detach())})
        return loss

    try:
        opt.step(closure)
        if sim.read(L.F_STATUS):
            raise RuntimeError("the fit drove the simulation into a flagged state")
    finally:
        sim.close()
    best = min(history, key=lambda h: h["loss"])
    return {"E": best["E"], "nu": best["nu"], "loss": best["loss"], "evals": len(history), "history": history}
