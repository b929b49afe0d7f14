"""The grid operation at tile staging (MPM_OPT_GRID_AT_STAGING): one launch
per substep, each particle pass applying the grid operation to the momentum
of its substep as it stages the 8^3 node-velocity tile.  Held to the oracle
(teacher-forced pairs of substeps, so the fused pass runs between them, at
2e-5 after two substeps; free runs of 200 substeps) at the slab's shipped
launch shape and full size, on the 1M-particle slab, with box tools, with
particles drifting several cells between sorts, with calls of one substep,
under graph replay, and against the per-phase launches (which keep a grid
kernel between particle passes).  With MPM_OPT_PERSISTENT the fused
substeps between sorts run as one persistent launch with a grid barrier
between substeps; the same checks run in that form (teacher-forced calls of
four substeps, so a run of two crosses a barrier), and a spin limit of one
forces the barrier's timeout from the host."""
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
    from paper_2402_01181_amd.sim import Sim
    return Sim, _lib


def _say(msg):
    print(msg, flush=True)


def _opts(L, block=256, item=128, sort_every=32, gas=1, slots=3, pers=0):
    return {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_BLOCK: block, L.OPT_ITEM: item, L.OPT_SORT_EVERY: sort_every,
            L.OPT_NODE_SLOTS: slots, L.OPT_GRID_AT_STAGING: gas, L.OPT_PERSISTENT: pers}


def _pairs(orc, sim, L, sc, env, calls, k=2):
    """Teacher-forced calls of k substeps against the oracle's k substeps
    from the same FP32 state, held to k per-substep tolerances; returns the
    largest error."""
    nt = len(sc.envs[env].tools)
    tol = k * TOL_SUBSTEP
    worst = 0.0
    for call in range(calls):
        o = oracle_sim_like(orc, sc, env)
        o.state = oracle_state_from_gpu(orc, sim, env)
        o.T[:nt] = sim.read(L.F_TOOL_T, env)
        o.s = sim.read(L.F_STEP, env)
        o.run(k, threads=oracle_threads())
        sim.step(k)
        x, v, C, F = sim.particles(env)
        e = max(rel_err(x, o.state.x, FLOORS["x"]), rel_err(v, o.state.v, FLOORS["v"]),
                rel_err(F, o.state.F, FLOORS["F"]))
        eC = rel_err(C, o.state.C, max(1.0, np.abs(o.state.C).max()))
        _say(f"  call {call}: err x/v/F {e:.2e}, C {eC:.2e}")
        worst = max(worst, e)
        assert e <= tol and eC <= 1e-4, (call, e, eC)
        np.testing.assert_allclose(sim.read(L.F_TOOL_T, env), o.T[:nt], rtol=1e-12)
    return worst


@pytest.mark.parametrize("pers", [0, 1])
def test_gas_slab_full_size_teacher_forced_and_free(gpu, orc, pers):
    """The 30K slab at its shipped launch shape with the grid at staging:
    200 free substeps against the oracle, then teacher-forced calls."""
    Sim, L = gpu
    S = 200
    k = 4 if pers else 2
    sc = scenes.slab_scene(substeps=S)
    _say(f"grid at staging (persistent {pers}): slab 30K, 256/128/32/3, {S} free substeps, "
         f"then 3 teacher-forced calls of {k}")
    sim = Sim(sc, options=_opts(L, pers=pers))
    sim.step(S)
    o = oracle_sim_like(orc, sc).run(S, threads=oracle_threads())
    assert_free_running(sim.particles()[0], o.state.x, sc.envs[0].x, "slab 200 substeps")
    np.testing.assert_allclose(sim.read(L.F_TOOL_T), o.T[:1], rtol=1e-12)
    assert sim.read(L.F_STEP) == S and sim.read(L.F_STATUS) == 0
    _pairs(orc, sim, L, sc, 0, 3, k)


@pytest.mark.parametrize("pers", [0, 1])
def test_gas_perturbed_cube_and_edge_shapes(gpu, orc, pers):
    """A perturbed state (velocities, affine C and strain) on the cube, with
    the smallest workgroup and item sizes and one-particle node steps."""
    Sim, L = gpu
    sc = scenes.cube_scene(seed=31)
    scenes.perturbed_state(np.random.default_rng(32), sc.envs[0], v_scale=0.05, C_scale=1.0, F_scale=0.01)
    for block, item, slots in ((64, 16, 1), (128, 48, 3), (256, 512, 3)):
        _say(f"grid at staging (persistent {pers}): perturbed cube, block {block}, item {item}, slots {slots}")
        sim = Sim(sc, options=_opts(L, block=block, item=item, sort_every=3, slots=slots, pers=pers))
        _pairs(orc, sim, L, sc, 0, 2, 4 if pers else 2)


def test_gas_large_slab_pairs(gpu, orc):
    """The 1,048,576-particle slab on 128^3 (768-particle items), sticky
    capsule: teacher-forced pairs after 20 free substeps."""
    Sim, L = gpu
    sc = scenes.large_slab_scene(substeps=40)
    _say("grid at staging: large slab 1M, 256/768/32/3, 20 free substeps then 2 teacher-forced pairs")
    sim = Sim(sc, options=_opts(L, item=768))
    sim.step(20)
    _pairs(orc, sim, L, sc, 0, 2)


def test_gas_box_gripper(gpu, orc):
    """Two box jaws (slip contact) instead of the capsule."""
    Sim, L = gpu
    sc = scenes.tool_slab_scene(seed=33, n_particles=6000, kind="gripper", n=32, substeps=10)
    _say("grid at staging: box gripper, 6000 particles on 32^3")
    sim = Sim(sc, options=_opts(L, sort_every=4))
    sim.step(4)
    _pairs(orc, sim, L, sc, 0, 3)


def test_gas_matches_per_phase_and_graph(gpu, orc):
    """Calls of 1, 2, 3, 40 and 40 substeps (sorts every 16, so sorts fall
    inside calls) with the grid at staging, eager and from a captured graph,
    against the per-phase launches; the node velocities the tail leaves for
    bricks holding particles match the grid kernel's."""
    Sim, L = gpu
    sc = scenes.slab_scene(seed=5, substeps=120)
    _say("grid at staging vs per-phase launches: slab 30K, calls 1, 2, 3, 40, 40")
    ref = Sim(sc, options=_opts(L, sort_every=16, gas=0))
    gas = Sim(sc, options=_opts(L, sort_every=16))
    gph = Sim(sc, options={**_opts(L, sort_every=16), L.OPT_GRAPH: 1})
    run = Sim(sc, options=_opts(L, sort_every=16, pers=1))
    rgph = Sim(sc, options={**_opts(L, sort_every=16, pers=1), L.OPT_GRAPH: 1})
    for n in (1, 2, 3, 40, 40):
        for s in (ref, gas, gph, run, rgph):
            s.step(n)
        xr, vr, _, Fr = ref.particles()
        for name, s in (("eager", gas), ("graph", gph), ("persistent", run), ("persistent graph", rgph)):
            x, v, _, F = s.particles()
            ex, ev, eF = np.abs(x - xr).max(), rel_err(v, vr, FLOORS["v"]), rel_err(F, Fr, FLOORS["F"])
            _say(f"  after a call of {n} ({name}): |dx| {ex:.2e}, v {ev:.2e}, F {eF:.2e}")
            assert ex <= 1e-5 and ev <= 1e-3 and eF <= 1e-3
            assert s.read(L.F_STATUS) == 0 and s.read(L.F_STEP) == ref.read(L.F_STEP)
            np.testing.assert_array_equal(s.read(L.F_TOOL_T), ref.read(L.F_TOOL_T))
    # node velocities of bricks that hold particles
    n = sc.envs[0].n
    x = gas.particles()[0]
    base = np.clip(np.floor(x * n - 0.5).astype(int), 0, n - 3) // 4
    bricks = np.unique(base[:, 0] * (n // 4) ** 2 + base[:, 1] * (n // 4) + base[:, 2])
    ijk = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    nb = ((ijk[:, 0] // 4) * (n // 4) + ijk[:, 1] // 4) * (n // 4) + ijk[:, 2] // 4
    mask = np.isin(nb, bricks)
    vg = gas.read(L.F_GRID_V, device=False)[:, mask]
    vr = ref.read(L.F_GRID_V, device=False)[:, mask]
    err = float(np.abs(vg - vr).max())
    _say(f"  grid velocities of {mask.sum()} nodes in occupied bricks: max |dv| {err:.2e}")
    assert err <= 1e-3 * max(1e-2, float(np.abs(vr).max()))
    assert np.abs(gas.read(L.F_GRID_M, device=False)).max() == 0.0   # every momentum buffer is clear after a call


@pytest.mark.parametrize("pers", [0, 1])
@pytest.mark.parametrize("sort_every,S", [(1000, 150), (50, 300)])
def test_gas_far_drift(gpu, orc, sort_every, S, pers):
    """A block translating rigidly at ~4.5 m/s (no gravity) moves several
    cells between sorts: its stencils leave the 8^3 tiles and reach bricks
    outside the static list (full clears of the momentum buffers they wrote).
    Closed form: x = x0 + S dt u, v = u, F = I."""
    Sim, L = gpu
    rng = np.random.default_rng(7)
    x = scenes.box_uniform(rng, 6000, (0.30, 0.30, 0.30), (0.45, 0.45, 0.45))
    v, C, F = scenes._rest_state(x)
    u = np.array([3.0, -2.0, 2.5], np.float32)
    v[:] = u
    env = scenes.Env(n=64, x=x, v=v, C=C, F=F, E=1e4, nu=0.3, rho=1e3, V0=0.15 ** 3 / x.shape[0])
    sc = scenes.Scene("drift", [env], dt=1e-4, substeps=S, gravity=(0.0, 0.0, 0.0))
    _say(f"grid at staging (persistent {pers}), far drift: {S} substeps, sort every {sort_every}")
    sim = Sim(sc, options=_opts(L, sort_every=sort_every, pers=pers))
    sim.step(S // 2)
    sim.step(S - S // 2)
    xt, vt, Ct, Ft = sim.particles()
    x_exact = env.x.astype(np.float64) + S * float(np.float32(sc.dt)) * u.astype(np.float64)
    ex, ev, eF = np.abs(xt - x_exact).max(), np.abs(vt - u).max(), np.abs(Ft - np.eye(3)).max()
    moved = np.abs(xt - env.x).max() * 64
    _say(f"  moved {moved:.2f} cells; |x - exact| {ex:.2e}, |v - u| {ev:.2e}, |F - I| {eF:.2e}")
    assert moved > 2.5 * S / 150
    assert ex <= 2e-5 * S / 150 and ev <= 1e-4 and eF <= 1e-5
    assert sim.read(L.F_STATUS) == 0 and sim.read(L.F_STEP) == S


def test_gas_run_barrier_timeout(gpu):
    """A spin limit of one makes the persistent run's grid barrier time out
    (forced from the host: every workgroup still leaves its bounded wait):
    the call returns with MPM_FLAG_BARRIER_TIMEOUT set.  With the default
    limit restored the same context runs on (the run resets its counters)
    and a fresh context stays clean."""
    Sim, L = gpu
    sc = scenes.slab_scene(seed=6, substeps=120)
    _say("persistent run, spin limit 1: 40 substeps")
    sim = Sim(sc, options={**_opts(L, sort_every=32, pers=1), L.OPT_SPIN_LIMIT: 1})
    sim.step(40)
    st = sim.read(L.F_STATUS)
    _say(f"  status {st}")
    assert st & L.FLAG_BARRIER_TIMEOUT
    sim.set_option(L.OPT_SPIN_LIMIT, 1 << 22)
    sim.step(40)
    assert np.isfinite(sim.particles()[0]).all()
    clean = Sim(sc, options=_opts(L, sort_every=32, pers=1))
    clean.step(40)
    assert clean.read(L.F_STATUS) == 0 and clean.read(L.F_STEP) == 40
