"""Helpers shared by the GPU parity tests: the error metric and oracle setup.

The metric is max|gpu - oracle| / max(max|oracle|, floor), with floors that
keep near-zero fields from being judged relatively (x: 1 m, v: 1e-2 m/s,
F: 1, grid momentum: 1e-2 * max grid mass).
"""
import numpy as np

TOL_SUBSTEP = 1e-5          # per substep, teacher-forced
TOL_DRIFT = 1e-3            # particle position after free running, fraction of the unit domain
# Free running, also: the position error must stay below this fraction of the
# largest displacement of the run, so the comparison means something when the
# tissue moves far less than 1e-3 m.  FP32 positions near 0.5 m round to
# ~3e-8 m per substep; over 200 substeps that is at most ~6e-6 m, under 1% of
# the sub-millimetre displacements of the benchmark scenes.
TOL_DISPLACEMENT = 2e-2
FLOORS = {"x": 1.0, "v": 1e-2, "F": 1.0, "C": 1.0}


def rel_err(gpu, ref, floor):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.abs(gpu - ref).max() / max(np.abs(ref).max(), floor))


def oracle_threads():
    """Threads for the oracle's threaded run (same result as serial): the
    host cores this process may use, at most 16."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def free_running_errors(x_gpu, x_oracle, x0):
    """(max position error, max displacement of the oracle's run) in metres."""
    x_gpu, x_oracle, x0 = (np.asarray(a, np.float64) for a in (x_gpu, x_oracle, x0))
    return float(np.abs(x_gpu - x_oracle).max()), float(np.abs(x_oracle - x0).max())


def assert_free_running(x_gpu, x_oracle, x0, what=""):
    err, disp = free_running_errors(x_gpu, x_oracle, x0)
    print(f"  {what} max |x - oracle| {err:.2e} m, max displacement {disp:.2e} m, ratio {err / max(disp, 1e-30):.2e}",
          flush=True)
    assert err <= TOL_DRIFT, (what, err)
    assert err <= TOL_DISPLACEMENT * disp, (what, err, disp)
    return err, disp


def oracle_state_from_gpu(orc, sim, env=0):
    """An oracle State holding exactly the GPU's current FP32 state."""
    x, v, C, F = sim.particles(env)
    f = lambda a: np.ascontiguousarray(a.astype(np.float64))
    return orc.State(f(x), f(v), f(C), f(F))


def oracle_sim_like(orc, scene, env_index=0):
    env = scene.envs[env_index]
    return orc.Sim(env, dt=scene.dt, gravity=scene.gravity, bound=scene.bound)
