"""Parity at the benchmark sizes, in the launch configuration the benchmark
uses (the autotuner's answer, which for these workloads is the shipped
MI355X table): the 1,048,576-particle slab on 128^3 and the 256-environment
batch.  The oracle computes what it can one by one: the large slab free
running and then teacher-forced substeps element by element;
for the batch, a seeded sample of environments, each free running and then
teacher-forced on its own.  Free runs last 200 substeps and are also held to
2% of the run's largest displacement (the tissue moves far less than the
1e-3 m domain bound in 200 substeps); the oracle runs threaded, which gives
its serial result bit for bit."""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes
from parity import (FLOORS, TOL_SUBSTEP, assert_free_running, oracle_sim_like, oracle_state_from_gpu, oracle_threads,
                    rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU")
    from paper_2402_01181_amd import _lib
    from paper_2402_01181_amd.autotune import autotune
    from paper_2402_01181_amd.sim import Sim
    return Sim, _lib, autotune


def _say(msg):
    print(msg, flush=True)


def _teacher_forced(orc, sim, L, sc, env, s0, steps):
    o = oracle_sim_like(orc, sc, env)
    nt = len(sc.envs[env].tools)
    worst = 0.0
    for s in range(s0, s0 + steps):
        o.state = oracle_state_from_gpu(orc, sim, env)
        o.T[:nt] = sim.read(L.F_TOOL_T, env)
        o.s = s
        o.run(1)
        sim.step(1)
        x, v, C, F = sim.particles(env)
        e = max(rel_err(x, o.state.x, FLOORS["x"]), rel_err(v, o.state.v, FLOORS["v"]),
                rel_err(F, o.state.F, FLOORS["F"]))
        worst = max(worst, e)
        assert e <= TOL_SUBSTEP, (env, s, e)
    return worst


def test_large_slab_full_size(gpu, orc):
    Sim, L, autotune = gpu
    S = 200
    sc = scenes.large_slab_scene(substeps=S + 2)
    opts = autotune(sc)
    _say(f"large slab 1,048,576 particles, 128^3, options {opts}: {S} free substeps, then 2 teacher-forced")
    sim = Sim(sc, options=opts)
    sim.step(S)
    o = oracle_sim_like(orc, sc).run(S, threads=oracle_threads())
    assert_free_running(sim.particles()[0], o.state.x, sc.envs[0].x, f"large slab {S} substeps")
    worst = _teacher_forced(orc, sim, L, sc, 0, S, 2)
    _say(f"  teacher-forced worst {worst:.2e}")
    assert sim.read(L.F_STATUS) == 0


def test_batched_full_size_sampled_environments(gpu, orc):
    Sim, L, autotune = gpu
    S = 200
    sc = scenes.batched_scene(substeps=S + 2)
    opts = autotune(sc)
    pick = np.random.default_rng(99).choice(len(sc.envs), 4, replace=False)
    _say(f"batch 256 environments, {sc.n_particles} particles, options {opts}: environments {pick.tolist()}, "
         f"{S} free substeps, then 2 teacher-forced")
    sim = Sim(sc, options=opts)
    sim.step(S)
    for e in pick:
        o = oracle_sim_like(orc, sc, int(e)).run(S, threads=oracle_threads())
        assert_free_running(sim.particles(int(e))[0], o.state.x, sc.envs[e].x,
                            f"env {e} (N {sc.envs[e].N}, {sc.envs[e].n}^3)")
    # teacher forcing steps every environment; check the sampled ones each substep
    for s in range(S, S + 2):
        orcs = {}
        for e in pick:
            o = oracle_sim_like(orc, sc, int(e))
            o.state = oracle_state_from_gpu(orc, sim, int(e))
            o.T[:1] = sim.read(L.F_TOOL_T, int(e))
            o.s = s
            orcs[int(e)] = o.run(1)
        sim.step(1)
        for e, o in orcs.items():
            x, v, C, F = sim.particles(e)
            err = max(rel_err(x, o.state.x, FLOORS["x"]), rel_err(v, o.state.v, FLOORS["v"]),
                      rel_err(F, o.state.F, FLOORS["F"]))
            assert err <= TOL_SUBSTEP, (e, s, err)
    assert all(sim.read(L.F_STATUS, e) == 0 for e in range(len(sc.envs)))
