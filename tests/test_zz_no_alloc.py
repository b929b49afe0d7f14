"""mpm_create_static (the entry point for callers that cannot allocate device
memory) against mpm_create with a caller-allocated workspace: the same scene
stepped through both must give the same particle state to the per-substep
tolerance, for two contexts in a row on the device's one static workspace,
the second smaller than the first (so it starts on the first one's leftovers)."""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes
from parity import FLOORS, TOL_SUBSTEP, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU")
    from paper_2402_01181_amd import _lib
    from paper_2402_01181_amd.sim import Sim
    return Sim, _lib


def _scene(n_particles, seed):
    sc = scenes.small_slab_scene(seed=seed, n_particles=n_particles, n=32, substeps=8, u=(0.05, -0.4, 0.02),
                                 dt=1e-4)
    tool = sc.envs[0].tools[0]
    tool.T0 = (tool.T0 - np.array([0.0, 0.015, 0.0])).astype(np.float32)   # pressing into the slab
    return sc


def _run(Sim, L, sc, static, steps):
    sim = Sim(sc, static_workspace=static,
              options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 4, L.OPT_ITEM: 128})
    sim.step(steps)
    out = sim.particles(0), sim.read(L.F_STATUS)
    sim.close()
    return out


@pytest.mark.parametrize("n_first,n_second", [(6000, 2500)])
def test_static_workspace_matches_caller_workspace(gpu, n_first, n_second):
    Sim, L = gpu
    steps = 6
    for call, (n, seed) in enumerate([(n_first, 11), (n_second, 12)]):
        print(f"no-alloc entry point, call {call + 1}: slab {n} particles, 32^3, {steps} substeps", flush=True)
        sc = _scene(n, seed)
        (xs, vs, Cs, Fs), st_s = _run(Sim, L, sc, True, steps)
        (xc, vc, Cc, Fc), st_c = _run(Sim, L, sc, False, steps)
        assert st_s == 0 and st_c == 0, (st_s, st_c)
        ex = rel_err(xs, xc, FLOORS["x"])
        ev = rel_err(vs, vc, FLOORS["v"])
        eF = rel_err(Fs, Fc, FLOORS["F"])
        eC = rel_err(Cs, Cc, max(1.0, np.abs(Cc).max()))
        moved = float(np.abs(xc - sc.envs[0].x).max())
        print(f"  static vs caller workspace: x {ex:.2e} v {ev:.2e} F {eF:.2e} C {eC:.2e}, moved {moved:.2e} m",
              flush=True)
        assert moved > 0
        assert ex <= TOL_SUBSTEP and ev <= TOL_SUBSTEP and eF <= TOL_SUBSTEP and eC <= 1e-4


def test_static_workspace_errors(gpu):
    Sim, L = gpu
    sim = Sim(_scene(2000, 13), static_workspace=True)
    with pytest.raises(L.MpmError) as e:
        Sim(_scene(1000, 14), static_workspace=True)        # the device's array is taken
    assert e.value.code == L.MPM_E_STATE
    sim.close()
    again = Sim(_scene(1000, 14), static_workspace=True)   # free again after destroy
    again.close()
    big = scenes.large_slab_scene(n_particles=1 << 20)
    with pytest.raises(L.MpmError) as e:
        Sim(big, static_workspace=True)                      # needs far more than the array holds
    assert e.value.code == L.MPM_E_WORKSPACE
