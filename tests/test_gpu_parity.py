"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Per stage and per substep the GPU starts from its own FP32 state and the
oracle from the same values promoted to FP64 (teacher forcing); errors use the
metric in parity.py against the per-substep tolerance 1e-5.  Free-running
runs are held to 1e-3 of the domain in particle position.
"""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes
from parity import (FLOORS, TOL_DRIFT, TOL_SUBSTEP, assert_free_running, oracle_sim_like, oracle_state_from_gpu,
                    oracle_threads, rel_err)

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


def _scheme(L, name):
    return {"direct": L.SCHEME_DIRECT, "tiled": L.SCHEME_TILED}[name]


def _perturbed_cube(seed=1):
    sc = scenes.cube_scene(seed=seed)
    scenes.perturbed_state(np.random.default_rng(seed + 100), sc.envs[0], v_scale=0.05, C_scale=1.0,
                           F_scale=0.01)
    return sc


def _compare_particles(orc_state, gpu_sim, env=0, tol=TOL_SUBSTEP, what=""):
    x, v, C, F = gpu_sim.particles(env)
    ex = rel_err(x, orc_state.x, FLOORS["x"])
    ev = rel_err(v, orc_state.v, FLOORS["v"])
    eF = rel_err(F, orc_state.F, FLOORS["F"])
    eC = rel_err(C, orc_state.C, max(1.0, np.abs(orc_state.C).max()))
    _say(f"  {what} err x={ex:.2e} v={ev:.2e} F={eF:.2e} C={eC:.2e}")
    assert ex <= tol and ev <= tol and eF <= tol, (what, ex, ev, eF)
    assert eC <= 1e-4, (what, eC)
    return ex, ev, eF


def test_stage_parity_cube(gpu, orc):
    Sim, L = gpu
    _say("stage parity: cube 8192 particles, 32^3, perturbed state")
    sc = _perturbed_cube()
    sim = Sim(sc)
    o = oracle_sim_like(orc, sc)
    o.state = oracle_state_from_gpu(orc, sim)
    sim.stage(L.STAGE_P2G)
    gm, gmv = o.p2g()
    m, mv, _ = sim.grid()
    em = rel_err(m, gm, 0.0)
    emv = rel_err(mv, gmv, 1e-2 * gm.max())
    _say(f"  P2G err m={em:.2e} mv={emv:.2e}")
    assert em <= TOL_SUBSTEP and emv <= TOL_SUBSTEP
    assert abs(m.astype(np.float64).sum() - gm.sum()) <= 1e-6 * gm.sum()    # mass conservation on the GPU
    sim.stage(L.STAGE_GRID)
    gv = o.grid_update(gm, gmv)
    _, _, v = sim.grid()
    ev = rel_err(v, gv, FLOORS["v"])
    _say(f"  GRID err v={ev:.2e}")
    assert ev <= TOL_SUBSTEP
    sim.stage(L.STAGE_G2P)
    o.g2p(gv)
    _compare_particles(o.state, sim, what="G2P")
    assert sim.read(L.F_STATUS) == 0


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
def test_substep_parity_slab_with_tool(gpu, orc, scheme):
    Sim, L = gpu
    for contact in (scenes.CONTACT_SLIP, scenes.CONTACT_STICKY):
        _say(f"substep parity ({scheme}): small slab 4000 particles, 32^3, contact={contact}")
        sc = scenes.small_slab_scene(seed=23, n_particles=4000, n=32, substeps=30, contact=contact,
                                     u=(0.05, -0.5, 0.0))
        sc.envs[0].tools[0].T0 = (sc.envs[0].tools[0].T0 - np.array([0, 0.012, 0])).astype(np.float32)
        sim = Sim(sc, options={L.OPT_SCHEME: _scheme(L, scheme), L.OPT_SORT_EVERY: 4})
        o = oracle_sim_like(orc, sc)
        worst = 0.0
        for s in range(sc.substeps):
            o.state = oracle_state_from_gpu(orc, sim)
            o.T[0] = sim.read(L.F_TOOL_T)[0]
            o.s = s
            o.run(1)
            sim.step(1)
            worst = max(worst, max(_compare_particles(o.state, sim, what=f"substep {s}")))
        np.testing.assert_allclose(sim.read(L.F_TOOL_T)[0], o.T[0], rtol=1e-12)
        assert sim.read(L.F_STEP) == sc.substeps
        _say(f"  worst {worst:.2e}")


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
def test_free_running_cube_200(gpu, orc, scheme):
    """The cube of configuration 1 settling under gravity on the sticky
    floor, 200 substeps in one call (sorts every 8), against the oracle; the
    error is also held to 2% of the largest displacement."""
    Sim, L = gpu
    _say(f"free running ({scheme}): cube 8192 particles, 200 substeps in one call, sort every 8")
    sc = scenes.cube_scene(seed=1, substeps=200)
    sim = Sim(sc, options={L.OPT_SCHEME: _scheme(L, scheme), L.OPT_SORT_EVERY: 8})
    sim.step(sc.substeps)
    o = oracle_sim_like(orc, sc).run(sc.substeps)
    x, v, C, F = sim.particles()
    assert_free_running(x, o.state.x, sc.envs[0].x, "cube 200 substeps")
    assert rel_err(v, o.state.v, FLOORS["v"]) <= 1e-2
    assert sim.read(L.F_STATUS) == 0


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
def test_free_running_slab_200(gpu, orc, scheme):
    """The 30K slab pressed by the capsule (slip, friction 0.3), 200
    substeps in calls of 120 and 80 at the benchmark's launch shapes."""
    Sim, L = gpu
    from paper_2402_01181_amd.autotune import autotune
    sc = scenes.slab_scene(seed=2, substeps=200)
    opts = autotune(sc) if scheme == "tiled" else {L.OPT_SCHEME: L.SCHEME_DIRECT}
    _say(f"free running ({scheme}): slab 30K, 200 substeps, options {opts}")
    sim = Sim(sc, options=opts)
    sim.step(120)
    sim.step(80)
    o = oracle_sim_like(orc, sc).run(sc.substeps, threads=oracle_threads())
    x, v, C, F = sim.particles()
    assert_free_running(x, o.state.x, sc.envs[0].x, "slab 200 substeps")
    np.testing.assert_allclose(sim.read(L.F_TOOL_T)[0], o.T[0], rtol=1e-12)
    assert sim.read(L.F_STATUS) == 0


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
def test_slab_30k_one_substep_full_size(gpu, orc, scheme):
    Sim, L = gpu
    _say(f"slab 30K, 64^3 ({scheme}): teacher-forced substeps at full size")
    sc = scenes.slab_scene(seed=2, substeps=5)
    scenes.perturbed_state(np.random.default_rng(5), sc.envs[0], v_scale=0.02, C_scale=0.5, F_scale=0.005)
    sim = Sim(sc, options={L.OPT_SCHEME: _scheme(L, scheme)})
    o = oracle_sim_like(orc, sc)
    for s in range(3):
        o.state = oracle_state_from_gpu(orc, sim)
        o.T[0] = sim.read(L.F_TOOL_T)[0]
        o.s = s
        o.run(1)
        sim.step(1)
        _compare_particles(o.state, sim, what=f"substep {s}")


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
def test_status_flags_and_read_errors(gpu, orc, scheme):
    Sim, L = gpu
    _say(f"status flags ({scheme})")
    sc = scenes.small_slab_scene(seed=3, n_particles=500, n=32, substeps=1)
    env = sc.envs[0]
    env.x[0] = [0.01, 0.5, 0.5]          # stencil leaves the grid
    env.F[1] = np.diag([1.0, 1.0, -0.5]).astype(np.float32)   # inverted
    sim = Sim(sc, options={L.OPT_SCHEME: _scheme(L, scheme)})
    sim.step(3)
    st = sim.read(L.F_STATUS)
    assert st & L.FLAG_OUT_OF_DOMAIN and st & L.FLAG_INVERTED
    x, v, C, F = sim.particles()
    np.testing.assert_array_equal(x[0], env.x[0])                # frozen particle
    import ctypes as ct
    buf = np.zeros(3, np.float32)
    assert sim.lib.mpm_read_state(sim.ctx, 0, L.F_X, buf.ctypes.data_as(ct.c_void_p), 12, 0, None) == L.MPM_E_ARG
    assert sim.lib.mpm_read_state(sim.ctx, 5, L.F_X, buf.ctypes.data_as(ct.c_void_p), 12, 0, None) == L.MPM_E_ARG
    assert sim.lib.mpm_set_tool(sim.ctx, 0, 3, None, None, 0) == L.MPM_E_ARG


@pytest.mark.parametrize("gas,persistent", [(0, 0), (1, 0), (1, 1), (0, 1)])
def test_frozen_state_kept_across_sorts_within_a_call(gpu, orc, gas, persistent):
    """Particles whose stencil leaves the grid are frozen (x, v, C, F
    unchanged, Sec. III-B: no transfer for them).  Between the fused substeps
    of a call only such particles carry v and C, and a sort there moves those
    two fields for particles near the domain edge alone: twelve substeps in
    one call, sorting every two, must leave every frozen particle's state
    exactly as it was, in each launch form."""
    Sim, L = gpu
    _say(f"frozen particles across sorts within a call (grid at staging {gas}, persistent {persistent})")
    sc = scenes.small_slab_scene(seed=6, n_particles=3000, n=32, substeps=12)
    env = sc.envs[0]
    rng = np.random.default_rng(11)
    frozen = [3, 70, 511, 1200, 2999]
    places = [[0.01, 0.5, 0.5], [0.5, 0.995, 0.5], [0.5, 0.2, 0.004], [0.99, 0.3, 0.6], [0.4, 0.001, 0.98]]
    for k, p in zip(frozen, places):
        env.x[k] = p
        env.v[k] = rng.uniform(-0.3, 0.3, 3)
        env.C[k] = rng.uniform(-2.0, 2.0, (3, 3))
        env.F[k] = np.eye(3) + rng.uniform(-0.02, 0.02, (3, 3))
    opts = {L.OPT_SORT_EVERY: 2, L.OPT_GRID_AT_STAGING: gas, L.OPT_PERSISTENT: persistent, L.OPT_ITEM: 128}
    sim = Sim(sc, options=opts)
    x0, v0, C0, F0 = (a.copy() for a in sim.particles())
    sim.step(12)
    assert sim.read(L.F_STATUS) & L.FLAG_OUT_OF_DOMAIN
    x, v, C, F = sim.particles()
    for k in frozen:
        np.testing.assert_array_equal(x[k], x0[k])
        np.testing.assert_array_equal(v[k], v0[k])
        np.testing.assert_array_equal(C[k], C0[k])
        np.testing.assert_array_equal(F[k], F0[k])
    moved = np.setdiff1d(np.arange(sc.n_particles), frozen)
    assert np.abs(x[moved] - x0[moved]).max() > 0.0     # the rest of the slab did step
    sim.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_frozen_state_kept_across_sorts_two_environments(gpu, orc, persistent):
    """The edge test of the sort between fused substeps with two
    environments of different grid sizes (the test looks each particle's
    environment up): frozen particles in both keep x, v, C and F exactly over
    twelve substeps sorted every two."""
    Sim, L = gpu
    _say(f"frozen particles across sorts, two environments (persistent {persistent})")
    a = scenes.small_slab_scene(seed=7, n_particles=2500, n=32, substeps=12)
    b = scenes.small_slab_scene(seed=8, n_particles=1800, n=24, substeps=12)
    sc = scenes.Scene("two-slabs", [a.envs[0], b.envs[0]], dt=a.dt, substeps=12)
    rng = np.random.default_rng(12)
    frozen = {0: [5, 900, 2499], 1: [0, 777, 1799]}
    places = [[0.01, 0.5, 0.5], [0.5, 0.997, 0.3], [0.6, 0.3, 0.002]]
    for e, ks in frozen.items():
        env = sc.envs[e]
        for k, p in zip(ks, places):
            env.x[k] = p
            env.v[k] = rng.uniform(-0.3, 0.3, 3)
            env.C[k] = rng.uniform(-2.0, 2.0, (3, 3))
    sim = Sim(sc, options={L.OPT_SORT_EVERY: 2, L.OPT_PERSISTENT: persistent, L.OPT_ITEM: 128})
    before = {e: [q.copy() for q in sim.particles(e)] for e in frozen}
    sim.step(12)
    for e, ks in frozen.items():
        assert sim.read(L.F_STATUS, e) & L.FLAG_OUT_OF_DOMAIN
        after = sim.particles(e)
        for k in ks:
            for q0, q1 in zip(before[e], after):
                np.testing.assert_array_equal(q1[k], q0[k])
    sim.close()


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
def test_nonfinite_flag(gpu, orc, scheme):
    """A particle given a NaN velocity makes its node momenta NaN; the G2P
    that follows gives NaN velocities and positions, which set
    MPM_FLAG_NONFINITE (a NaN position then counts as outside the grid: the
    particle is frozen and no index is formed from it)."""
    Sim, L = gpu
    _say(f"non-finite flag ({scheme})")
    sc = scenes.small_slab_scene(seed=4, n_particles=500, n=32, substeps=1)
    sc.envs[0].v[7] = [np.nan, 0.0, 0.0]
    sim = Sim(sc, options={L.OPT_SCHEME: _scheme(L, scheme), L.OPT_SORT_EVERY: 2})
    sim.step(4)
    st = sim.read(L.F_STATUS)
    _say(f"  status {st:#x}")
    assert st & L.FLAG_NONFINITE
    x = sim.particles()[0]
    assert not np.isfinite(x[7]).all()
    # a clean scene raises nothing
    clean = Sim(scenes.small_slab_scene(seed=4, n_particles=500, n=32, substeps=1),
                options={L.OPT_SCHEME: _scheme(L, scheme)})
    clean.step(4)
    assert clean.read(L.F_STATUS) == 0


@pytest.mark.parametrize("field,value", [("E", 0.0), ("E", float("nan")), ("E", float("inf")), ("nu", 0.5),
                                         ("nu", -1.0), ("nu", float("nan")), ("rho", 0.0), ("V0", -1.0)])
def test_material_validation(gpu, orc, field, value):
    """mpm_create reads the material table and refuses E <= 0 or non-finite,
    nu outside (-1, 0.5), rho <= 0 and V0 <= 0 with MPM_E_ARG."""
    Sim, L = gpu
    sc = scenes.small_slab_scene(seed=5, n_particles=200, n=16, substeps=1)
    setattr(sc.envs[0], field, value)
    with pytest.raises(L.MpmError) as e:
        Sim(sc)
    assert e.value.code == L.MPM_E_ARG
    assert "material" in str(e.value)


@pytest.mark.parametrize("slots", [1, 3])
def test_tiled_matches_direct_long_run(gpu, orc, slots):
    """Cross-check of the two schemes (different accumulation orders) on the
    30K slab with the tool pushing: 200 substeps, several sorts, mid-call,
    with either node-pass form."""
    Sim, L = gpu
    _say(f"tiled (node slots {slots}) vs direct: slab 30K, 200 substeps")
    sc = scenes.slab_scene(seed=2, substeps=200)
    a = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_DIRECT})
    b = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 16, L.OPT_NODE_SLOTS: slots})
    a.step(120)
    a.step(80)
    b.step(120)
    b.step(80)
    xa, va, Ca, Fa = a.particles()
    xb, vb, Cb, Fb = b.particles()
    ex = np.abs(xa - xb).max()
    ev = rel_err(vb, va, FLOORS["v"])
    _say(f"  max |dx| = {ex:.2e}, v err = {ev:.2e}")
    assert ex <= 1e-5 and ev <= 1e-3
    assert a.read(L.F_STATUS) == 0 and b.read(L.F_STATUS) == 0
    np.testing.assert_allclose(a.read(L.F_TOOL_T), b.read(L.F_TOOL_T), rtol=0, atol=0)


def test_graph_replays_match_eager(gpu, orc):
    """MPM_OPT_GRAPH: a captured 40-substep call replayed four times, with
    reads and syncs between replays, against the same calls run eagerly."""
    Sim, L = gpu
    import torch
    _say("graph replay vs eager: slab 30K, 4 x 40 substeps")
    sc = scenes.slab_scene(seed=2, substeps=160)
    eager = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 16})
    graph = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 16, L.OPT_GRAPH: 1})
    for r in range(4):
        eager.step(40)
        graph.step(40)
        torch.cuda.synchronize()
        xe, ve, _, _ = eager.particles()
        xg, vg, _, _ = graph.particles()
        ex = np.abs(xe - xg).max()
        ev = rel_err(vg, ve, FLOORS["v"])
        _say(f"  replay {r}: max |dx| = {ex:.2e}, v err = {ev:.2e}")
        assert ex <= 1e-5 and ev <= 1e-3
        assert graph.read(L.F_STEP) == 40 * (r + 1)
        np.testing.assert_array_equal(graph.read(L.F_TOOL_T), eager.read(L.F_TOOL_T))
    assert graph.read(L.F_STATUS) == 0


def _small_batch(seed=4, n_envs=6):
    return scenes.batched_scene(seed=seed, n_envs=n_envs, substeps=30, n_min=1500, n_max=5000)


def test_batched_matches_single_environments(gpu, orc):
    """Environments stepped together (one context, shared kernels) give the
    same trajectories as each environment stepped alone."""
    Sim, L = gpu
    sc = _small_batch()
    _say(f"batched vs single: {len(sc.envs)} envs, grids {[e.n for e in sc.envs]}, N {[e.N for e in sc.envs]}")
    b = Sim(sc, options={L.OPT_SORT_EVERY: 8})
    b.step(sc.substeps)
    for e, env in enumerate(sc.envs):
        one = scenes.Scene(f"env{e}", [env], dt=sc.dt, substeps=sc.substeps)
        s = Sim(one, options={L.OPT_SORT_EVERY: 8})
        s.step(sc.substeps)
        xb = b.particles(e)[0]
        xs = s.particles(0)[0]
        err = np.abs(xb - xs).max()
        _say(f"  env {e}: max |dx| = {err:.2e}")
        assert err <= 1e-5
        np.testing.assert_array_equal(b.read(L.F_TOOL_T, e), s.read(L.F_TOOL_T, 0))
        assert b.read(L.F_STEP, e) == sc.substeps and b.read(L.F_STATUS, e) == 0


def test_batched_teacher_forced_parity(gpu, orc):
    Sim, L = gpu
    sc = _small_batch(seed=9, n_envs=5)
    _say(f"batched teacher-forced parity: {len(sc.envs)} envs")
    b = Sim(sc)
    for s in range(3):
        refs = []
        for e, env in enumerate(sc.envs):
            o = orc.Sim(env, dt=sc.dt, gravity=sc.gravity, bound=sc.bound)
            o.state = oracle_state_from_gpu(orc, b, e)
            o.T[0] = b.read(L.F_TOOL_T, e)[0]
            o.s = s
            o.run(1)
            refs.append(o.state)
        b.step(1)
        for e, ref in enumerate(refs):
            _compare_particles(ref, b, env=e, what=f"substep {s} env {e}")


@pytest.mark.parametrize("use_graph", [0, 1])
def test_persistent_matches_eager(gpu, orc, use_graph):
    """MPM_OPT_PERSISTENT: runs of up to sort_every substeps in one kernel (one
    environment, so one group of workgroups); 3 calls of 40 substeps (runs of 16, 16, 8) against the
    same calls launched per phase.  No barrier may time out."""
    Sim, L = gpu
    _say(f"persistent (graph={use_graph}) vs eager: slab 30K, 3 x 40 substeps")
    sc = scenes.slab_scene(seed=3, substeps=120)
    opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 16}
    eager = Sim(sc, options=dict(opts))
    pers = Sim(sc, options={**opts, L.OPT_PERSISTENT: 1, L.OPT_GRAPH: use_graph})
    for r in range(3):
        eager.step(40)
        pers.step(40)
        assert pers.read(L.F_STATUS) == 0, "barrier timeout or other status flag"
        xe, ve, _, Fe = eager.particles()
        xp, vp, _, Fp = pers.particles()
        ex = np.abs(xe - xp).max()
        ev = rel_err(vp, ve, FLOORS["v"])
        eF = rel_err(Fp, Fe, FLOORS["F"])
        _say(f"  call {r}: max |dx| = {ex:.2e}, v err = {ev:.2e}, F err = {eF:.2e}")
        assert ex <= 1e-5 and ev <= 1e-3 and eF <= 1e-3
        assert pers.read(L.F_STEP) == 40 * (r + 1)
        np.testing.assert_array_equal(pers.read(L.F_TOOL_T), eager.read(L.F_TOOL_T))


def test_persistent_batched_and_single_substeps(gpu, orc):
    """Persistent form on a batch of environments, with calls of 1, 7 and
    22 substeps (a run of one substep, runs ending in the G2P tail)."""
    Sim, L = gpu
    sc = _small_batch(seed=5, n_envs=6)
    _say(f"persistent batched: {len(sc.envs)} envs, calls 1, 7, 22")
    eager = Sim(sc, options={L.OPT_SORT_EVERY: 8})
    pers = Sim(sc, options={L.OPT_SORT_EVERY: 8, L.OPT_PERSISTENT: 1})
    for n in (1, 7, 22):
        eager.step(n)
        pers.step(n)
    for e in range(len(sc.envs)):
        xe = eager.particles(e)[0]
        xp = pers.particles(e)[0]
        err = np.abs(xe - xp).max()
        _say(f"  env {e}: max |dx| = {err:.2e}")
        assert err <= 1e-5
        assert pers.read(L.F_STATUS, e) == 0 and pers.read(L.F_STEP, e) == 30
        np.testing.assert_array_equal(pers.read(L.F_TOOL_T, e), eager.read(L.F_TOOL_T, e))


def _many_small_envs(n_envs=700, seed=21):
    """n_envs slabs of 100-300 particles on 16^3 grids, each pressed by its own
    capsule: more environments than the persistent kernel has workgroups at
    256 threads, so workgroups step several environments each."""
    rng = np.random.default_rng(seed)
    envs = []
    for _ in range(n_envs):
        N = int(rng.integers(100, 301))
        y0 = 3.0 / 16
        x = scenes.box_uniform(rng, N, (0.25, y0, 0.25), (0.75, y0 + 0.15, 0.75))
        v, C, F = scenes._rest_state(x)
        u = rng.uniform(0.05, 0.2) * scenes._unit((rng.uniform(-0.3, 0.3), -1.0, rng.uniform(-0.3, 0.3)))
        tool = scenes.capsule_tool(T0=(0.5, y0 + 0.16, 0.5), u=u, radius=0.03, friction=0.3)
        envs.append(scenes.Env(n=16, x=x, v=v, C=C, F=F, E=float(rng.uniform(3e3, 3e4)),
                               nu=float(rng.uniform(0.25, 0.45)), rho=1e3, V0=0.5 * 0.15 * 0.5 / N, tools=[tool]))
    return scenes.Scene(f"many-{n_envs}", envs, dt=1e-4, substeps=30)


def test_persistent_more_envs_than_workgroups(gpu, orc):
    """Persistent form with 700 environments at 256 threads per workgroup
    (fewer co-resident workgroups than environments): calls of 1, 9 and 20
    substeps against the per-phase launches, then one teacher-forced pair of
    substeps of three environments against the oracle."""
    Sim, L = gpu
    sc = _many_small_envs()
    opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 8, L.OPT_BLOCK: 256, L.OPT_ITEM: 128}
    _say(f"persistent, {len(sc.envs)} environments of 100-300 particles on 16^3, calls 1, 9, 20")
    eager = Sim(sc, options=dict(opts))
    pers = Sim(sc, options={**opts, L.OPT_PERSISTENT: 1})
    for n in (1, 9, 20):
        eager.step(n)
        pers.step(n)
    worst = 0.0
    for e in range(len(sc.envs)):
        xe, xp = eager.particles(e)[0], pers.particles(e)[0]
        worst = max(worst, float(np.abs(xe - xp).max()))
        assert pers.read(L.F_STATUS, e) == 0 and pers.read(L.F_STEP, e) == 30
        np.testing.assert_array_equal(pers.read(L.F_TOOL_T, e), eager.read(L.F_TOOL_T, e))
    moved = max(float(np.abs(pers.particles(e)[0] - sc.envs[e].x).max()) for e in (0, 350, 699))
    _say(f"  max |x_persistent - x_eager| over all environments {worst:.2e} m (moved up to {moved:.2e} m)")
    assert worst <= 1e-5 and moved > 0
    refs = {}
    for e in (0, 350, 699):
        o = oracle_sim_like(orc, sc, e)
        o.state = oracle_state_from_gpu(orc, pers, e)
        o.T[:1] = pers.read(L.F_TOOL_T, e)
        o.s = pers.read(L.F_STEP, e)
        refs[e] = o.run(2)
    pers.step(2)
    for e, o in refs.items():
        _compare_particles(o.state, pers, env=e, tol=2 * TOL_SUBSTEP, what=f"env {e} two substeps")


@pytest.mark.parametrize("persistent,use_graph", [(1, 0), (1, 1), (0, 1)])
def test_batch_forms_against_oracle(gpu, orc, persistent, use_graph):
    """The batched forms checked against the oracle itself: the persistent
    kernel (runs of sort_every substeps, a barrier per environment group), with or without an
    internally captured graph, and the captured graph of per-phase launches.
    Each environment is teacher-forced over calls of two substeps (the fused
    particle pass runs between the two grid operations; 2e-5 after two
    substeps), then free-runs 200 substeps in calls of 100 against its own
    oracle run."""
    Sim, L = gpu
    sc = scenes.batched_scene(seed=12, n_envs=6, substeps=200, n_min=1500, n_max=5000)
    rng = np.random.default_rng(13)
    for env in sc.envs:
        scenes.perturbed_state(rng, env, v_scale=0.02, C_scale=0.5, F_scale=0.005)
    _say(f"batch forms vs oracle: persistent={persistent} graph={use_graph}, {len(sc.envs)} envs, "
         f"N {[e.N for e in sc.envs]}, grids {[e.n for e in sc.envs]}")
    opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 8, L.OPT_PERSISTENT: persistent, L.OPT_GRAPH: use_graph}
    sim = Sim(sc, options=opts)
    for call in range(3):
        refs = []
        for e, env in enumerate(sc.envs):
            o = oracle_sim_like(orc, sc, e)
            o.state = oracle_state_from_gpu(orc, sim, e)
            o.T[:1] = sim.read(L.F_TOOL_T, e)
            o.s = sim.read(L.F_STEP, e)
            refs.append(o.run(2))
        sim.step(2)
        for e, o in enumerate(refs):
            _compare_particles(o.state, sim, env=e, tol=2 * TOL_SUBSTEP, what=f"call {call} env {e}")
            assert sim.read(L.F_STATUS, e) == 0
    free = Sim(sc, options=opts)
    free.step(100)
    free.step(100)
    for e, env in enumerate(sc.envs):
        o = oracle_sim_like(orc, sc, e).run(200)
        assert_free_running(free.particles(e)[0], o.state.x, env.x, f"env {e} 200 substeps")
        np.testing.assert_allclose(free.read(L.F_TOOL_T, e)[0], o.T[0], rtol=1e-12)
        assert free.read(L.F_STATUS, e) == 0 and free.read(L.F_STEP, e) == 200


def _drift_scene(substeps=150):
    """A block translating rigidly at ~4.5 m/s with no gravity, far from the
    walls: in 150 substeps of 1e-4 s it moves ~2.9 cells of the 64^3 grid."""
    rng = np.random.default_rng(7)
    x = scenes.box_uniform(rng, 6000, (0.30, 0.30, 0.30), (0.45, 0.45, 0.45))
    v, C, F = scenes._rest_state(x)
    u = np.array([3.0, -2.0, 2.5], np.float32)
    v[:] = u
    env = scenes.Env(n=64, x=x, v=v, C=C, F=F, E=1e4, nu=0.3, rho=1e3, V0=0.15 ** 3 / x.shape[0])
    return scenes.Scene("drift", [env], dt=1e-4, substeps=substeps, gravity=(0.0, 0.0, 0.0)), u


@pytest.mark.parametrize("persistent,sort_every,S", [(0, 1000, 150), (1, 1000, 150), (0, 50, 300), (1, 50, 300)])
def test_far_drift_between_sorts(gpu, orc, persistent, sort_every, S):
    """Particles that move several cells past their sort-time brick reach
    bricks outside the static brick list; the dynamic lists must carry them.
    With one sort for the whole run, or a sort every 50 substeps, which in
    the persistent form falls between two runs, right after a P2G that listed
    far bricks (the next static list must take those bricks over).  Rigid
    translation has a closed form (x = x0 + S dt u, v = u, F = I) and the
    direct scheme keeps no lists."""
    Sim, L = gpu
    sc, u = _drift_scene(S)
    _say(f"far drift: 6000 particles, {S} substeps in one call, sort every {sort_every}, persistent={persistent}")
    tiled = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: sort_every,
                             L.OPT_PERSISTENT: persistent})
    direct = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_DIRECT})
    tiled.step(S)
    direct.step(S)
    xt, vt, Ct, Ft = tiled.particles()
    xd, _, _, _ = direct.particles()
    x_exact = sc.envs[0].x.astype(np.float64) + S * float(np.float32(sc.dt)) * u.astype(np.float64)
    moved = np.abs(xt - sc.envs[0].x).max() * 64
    ex = np.abs(xt - x_exact).max()
    ev = np.abs(vt - u).max()
    eF = np.abs(Ft - np.eye(3)).max()
    etd = np.abs(xt - xd).max()
    _say(f"  moved {moved:.2f} cells; |x - exact| {ex:.2e}, |v - u| {ev:.2e}, |F - I| {eF:.2e}, |tiled - direct| {etd:.2e}")
    assert moved > 2.5 * S / 150
    assert ex <= 2e-5 * S / 150 and ev <= 1e-4 and eF <= 1e-5 and etd <= 1e-5
    assert tiled.read(L.F_STATUS) == 0 and tiled.read(L.F_STEP) == S


@pytest.mark.parametrize("scheme", ["tiled", "direct"])
def test_largest_grid_free_fall(gpu, orc, scheme):
    """The largest grid (512^3, 134M nodes): a block at rest in free fall far
    from the walls moves rigidly, x = x0 + dt^2 g S(S+1)/2, v = S dt g,
    F = I (the substep's symplectic Euler with affine-exact transfers)."""
    Sim, L = gpu
    rng = np.random.default_rng(12)
    x = scenes.box_uniform(rng, 20000, (0.40, 0.40, 0.40), (0.45, 0.45, 0.45))
    v, C, F = scenes._rest_state(x)
    env = scenes.Env(n=512, x=x, v=v, C=C, F=F, E=1e4, nu=0.3, rho=1e3, V0=0.05 ** 3 / x.shape[0])
    S = 20
    sc = scenes.Scene("free-fall-512", [env], dt=1e-4, substeps=S)
    _say(f"largest grid ({scheme}): 20,000 particles on 512^3, {S} substeps of free fall")
    sim = Sim(sc, options={L.OPT_SCHEME: _scheme(L, scheme), L.OPT_SORT_EVERY: 8})
    sim.step(S)
    xt, vt, Ct, Ft = sim.particles()
    dt, g = float(np.float32(sc.dt)), np.array(sc.gravity, np.float64)
    x_exact = x.astype(np.float64) + dt * dt * g * S * (S + 1) / 2
    ex, ev = np.abs(xt - x_exact).max(), np.abs(vt - S * dt * g).max()
    eF, eC = np.abs(Ft - np.eye(3)).max(), np.abs(Ct).max()
    _say(f"  |x - exact| {ex:.2e}, |v - exact| {ev:.2e}, |F - I| {eF:.2e}, |C| {eC:.2e}")
    assert ex <= 1e-6 and ev <= 1e-5 and eF <= 1e-5 and eC <= 1e-3
    assert sim.read(L.F_STATUS) == 0 and sim.read(L.F_STEP) == S


def _ragged_scene(seed=11):
    """Three small environments of ragged sizes: one particle on an 8^3 grid,
    17 particles on a 12^3 grid, 300 in a cube on a 16^3 grid, all moving."""
    rng = np.random.default_rng(seed)
    envs = []
    for n, N, lo, hi in ((8, 1, 0.45, 0.55), (12, 17, 0.35, 0.65), (16, 300, 0.3, 0.6)):
        x = scenes.box_uniform(rng, N, (lo,) * 3, (hi,) * 3)
        v, C, F = scenes._rest_state(x)
        env = scenes.Env(n=n, x=x, v=v, C=C, F=F, E=3e3, nu=0.3, rho=1e3, V0=(hi - lo) ** 3 / N)
        scenes.perturbed_state(rng, env, v_scale=0.2, C_scale=1.0, F_scale=0.01)
        envs.append(env)
    return scenes.Scene("ragged", envs, dt=1e-4, substeps=20)


@pytest.mark.parametrize("block,item,slots", [(64, 16, 3), (256, 4096, 1), (128, 48, 3), (256, 128, 1)])
def test_ragged_tiny_environments(gpu, orc, block, item, slots):
    """Edge shapes: a one-particle environment, the smallest grid (8^3), item
    sizes from 16 to 4096 particles and workgroups of 64 to 256 threads; every
    environment free-runs 20 substeps against the oracle."""
    Sim, L = gpu
    sc = _ragged_scene()
    _say(f"ragged tiny envs: N {[e.N for e in sc.envs]}, grids {[e.n for e in sc.envs]}, block {block}, item {item}, "
         f"slots {slots}")
    sim = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_BLOCK: block, L.OPT_ITEM: item, L.OPT_SORT_EVERY: 7,
                           L.OPT_NODE_SLOTS: slots})
    sim.step(13)
    sim.step(7)
    for e, env in enumerate(sc.envs):
        o = orc.Sim(env, dt=sc.dt, gravity=sc.gravity, bound=sc.bound).run(sc.substeps)
        x, v, C, F = sim.particles(e)
        ex = np.abs(x - o.state.x).max()
        ev = rel_err(v, o.state.v, FLOORS["v"])
        _say(f"  env {e}: |dx| {ex:.2e}, v err {ev:.2e}")
        assert ex <= 1e-5 and ev <= 1e-4
        assert sim.read(L.F_STATUS, e) == 0 and sim.read(L.F_STEP, e) == sc.substeps


def test_autotune_picks_and_caches(gpu, orc, tmp_path):
    """The autotuner times its candidates, returns one of them, and a second
    call is answered from the JSON cache."""
    Sim, L = gpu
    from paper_2402_01181_amd.autotune import autotune, workload_key
    import json
    sc = scenes.cube_scene(seed=1, substeps=10)
    cache = str(tmp_path / "tune.json")
    kw = dict(substeps=8, warmup=2, cache=cache, blocks=(64, 256), items=(64, 512), sort_every=(8, 16),
              graph=(0, 1), persistent=(0,), slots=(3,), grid_at_staging=(0, 1), use_shipped=False)
    best = autotune(sc, **kw)
    _say(f"autotune cube: {best}")
    assert best[L.OPT_BLOCK] in (64, 256) and best[L.OPT_ITEM] in (64, 512) and best[L.OPT_SORT_EVERY] in (8, 16)
    table = json.load(open(cache))
    entry = table[workload_key(sc)]
    assert len(entry["trials"]) == 4 + 2 + 2 + 2
    assert autotune(sc, **kw) == best
    s = Sim(sc, options=best)   # the options are accepted by the library
    s.step(10)
    assert s.read(L.F_STATUS) == 0


def test_caller_captured_graph(gpu, orc):
    """mpm_substep issues only kernel launches and never synchronises, so a
    caller can capture it in its own graph (here torch.cuda.graph): a
    captured 16-substep call (with a sort inside) replayed five times, with
    reads and eager work between the replays, against eager calls."""
    Sim, L = gpu
    import torch
    _say("caller-captured graph: small slab 4000 particles, 32^3, 5 replays of 16 substeps")
    sc = scenes.small_slab_scene(seed=31, n_particles=4000, n=32, substeps=96, u=(0.0, -0.5, 0.0))
    opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 8}
    eager = Sim(sc, options=opts)
    capt = Sim(sc, options=opts)
    eager.step(16)
    capt.step(16)                      # warm: work items exist before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            capt.step(16)              # recorded, not run
    torch.cuda.synchronize()
    for r in range(5):
        g.replay()
        eager.step(16)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum().item()   # unrelated eager work between replays
        xe, xc = eager.particles()[0], capt.particles()[0]
        err = np.abs(xe - xc).max()
        _say(f"  replay {r}: max |dx| = {err:.2e}")
        assert err <= 1e-5 and np.isfinite(junk)
        assert capt.read(L.F_STEP) == 16 * (r + 2)
        np.testing.assert_array_equal(capt.read(L.F_TOOL_T), eager.read(L.F_TOOL_T))
    o = oracle_sim_like(orc, sc).run(96)
    assert_free_running(capt.particles()[0], o.state.x, sc.envs[0].x, "captured replays, 96 substeps")
    assert capt.read(L.F_STATUS) == 0
