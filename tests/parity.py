"""Helpers shared by the GPU parity tests: the error metric and oracle setup.

The metric is max|gpu - oracle| / max(max|oracle|, floor), with floors that
keep near-zero fields from being judged relatively (x: 1 m, v: 1e-2 m/s,
F: 1, grid momentum: 1e-2 * max grid mass).
"""
import numpy as np

TOL_SUBSTEP = 1e-5          # per substep, teacher-forced
TOL_DRIFT = 1e-3            # particle position after free running, fraction of the unit domain
FLOORS = {"x": 1.0, "v": 1e-2, "F": 1.0, "C": 1.0}


def rel_err(gpu, ref, floor):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.abs(gpu - ref).max() / max(np.abs(ref).max(), floor))


def oracle_state_from_gpu(orc, sim, env=0):
    """An oracle State holding exactly the GPU's current FP32 state."""
    x, v, C, F = sim.particles(env)
    f = lambda a: np.ascontiguousarray(a.astype(np.float64))
    return orc.State(f(x), f(v), f(C), f(F))


def oracle_sim_like(orc, scene, env_index=0):
    env = scene.envs[env_index]
    return orc.Sim(env, dt=scene.dt, gravity=scene.gravity, bound=scene.bound)
