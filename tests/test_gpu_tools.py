"""Box tools (gripper jaws) and sampled-SDF tools (Sec. III-C) on the GPU,
through the C ABI, against the FP64 oracle: the grid operation alone, every
substep teacher-forced (<= 1e-5), free running (<= 1e-3 of the domain), the
adjoint (<= 1e-3 of the oracle's adjoint) and argument checking."""
import ctypes as ct

import numpy as np
import pytest

from paper_2402_01181_amd import scenes
from parity import FLOORS, TOL_DRIFT, TOL_SUBSTEP, assert_free_running, oracle_sim_like, oracle_state_from_gpu, rel_err

pytestmark = pytest.mark.gpu

KINDS = [("gripper", scenes.SDF_TRILINEAR), ("sdf", scenes.SDF_TRILINEAR), ("sdf", scenes.SDF_NEAREST),
         ("mixed", scenes.SDF_TRILINEAR)]
KIND_IDS = ["gripper", "sdf-trilinear", "sdf-nearest", "mixed"]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU")
    from paper_2402_01181_amd import _lib
    from paper_2402_01181_amd.sim import Sim
    return Sim, _lib, torch


def _say(msg):
    print(msg, flush=True)


def _scene(kind, interp, N=4000, n=32, S=20, seed=61, contact=scenes.CONTACT_SLIP, perturb=False):
    sc = scenes.tool_slab_scene(seed, N, kind, n=n, substeps=S, sdf_res=48, interp=interp, contact=contact)
    if perturb:
        scenes.perturbed_state(np.random.default_rng(seed + 3), sc.envs[0], v_scale=0.05, C_scale=1.0, F_scale=0.01)
    return sc


@pytest.mark.parametrize("kind,interp", KINDS, ids=KIND_IDS)
def test_grid_operation_parity(gpu, orc, kind, interp):
    Sim, L, _ = gpu
    _say(f"grid operation parity: {kind} interp={interp}, 4000 particles, 32^3, perturbed state")
    sc = _scene(kind, interp, perturb=True)
    sim = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_DIRECT})
    o = oracle_sim_like(orc, sc)
    o.state = oracle_state_from_gpu(orc, sim)
    sim.stage(L.STAGE_P2G)
    gm, gmv = o.p2g()
    sim.stage(L.STAGE_GRID)
    gv, rec = o.grid_update(gm, gmv, record=True)
    tools = np.array([r.tool for r in rec])
    counts = [int((tools == t).sum()) for t in range(len(sc.envs[0].tools))]
    _say(f"  contact nodes per tool {counts}")
    assert all(c > 0 for c in counts)
    _, _, v = sim.grid()
    ev = rel_err(v, gv, FLOORS["v"])
    _say(f"  GRID err v={ev:.2e}")
    assert ev <= TOL_SUBSTEP


@pytest.mark.parametrize("scheme", ["direct", "tiled"])
@pytest.mark.parametrize("kind,interp", KINDS, ids=KIND_IDS)
def test_substep_parity_tools(gpu, orc, scheme, kind, interp):
    Sim, L, _ = gpu
    for contact in (scenes.CONTACT_SLIP, scenes.CONTACT_STICKY):
        _say(f"substep parity ({scheme}): {kind} interp={interp} contact={contact}, 4000 particles, 32^3, 20 substeps")
        sc = _scene(kind, interp, contact=contact)
        sim = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED if scheme == "tiled" else L.SCHEME_DIRECT,
                               L.OPT_SORT_EVERY: 4})
        o = oracle_sim_like(orc, sc)
        nt = len(sc.envs[0].tools)
        worst = 0.0
        for s in range(sc.substeps):
            o.state = oracle_state_from_gpu(orc, sim)
            o.T[:nt] = sim.read(L.F_TOOL_T)
            o.s = s
            o.run(1)
            sim.step(1)
            x, v, C, F = sim.particles()
            e = max(rel_err(x, o.state.x, FLOORS["x"]), rel_err(v, o.state.v, FLOORS["v"]),
                    rel_err(F, o.state.F, FLOORS["F"]))
            worst = max(worst, e)
            assert e <= TOL_SUBSTEP, (s, e)
        # the pose recurrence is the same FP64 arithmetic on both sides
        np.testing.assert_array_equal(sim.read(L.F_TOOL_T), o.T[:nt])
        assert sim.read(L.F_STATUS) == 0
        _say(f"  worst {worst:.2e}")


@pytest.mark.parametrize("kind,interp", KINDS, ids=KIND_IDS)
def test_free_running_tools(gpu, orc, kind, interp):
    Sim, L, _ = gpu
    S = 200
    _say(f"free running (tiled, graph): {kind} interp={interp}, 4000 particles, 32^3, {S} substeps, sort every 16")
    sc = _scene(kind, interp, S=S)
    sim = Sim(sc, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 16, L.OPT_GRAPH: 1})
    sim.step(S // 2)
    sim.step(S // 2)
    o = oracle_sim_like(orc, sc).run(S)
    x = sim.particles()[0]
    assert_free_running(x, o.state.x, sc.envs[0].x, f"{kind} {S} substeps")
    assert sim.read(L.F_STATUS) == 0


def test_switching_tool_shapes_recaptures_graph(gpu, orc):
    """A captured graph made with analytic tools only is not replayed once a
    sampled-SDF tool is set (its grid kernel has no SDF branch)."""
    Sim, L, _ = gpu
    _say("graph after switching a capsule slot to a sampled SDF: 4000 particles, 32^3")
    sc = _scene("sdf", scenes.SDF_TRILINEAR, S=16)
    probe = sc.envs[0].tools[0]
    capsule = scenes.capsule_tool(T0=probe.T0, u=probe.traj[0])
    sc_caps = _scene("sdf", scenes.SDF_TRILINEAR, S=16)
    sc_caps.envs[0].tools = [capsule]
    sim = Sim(sc_caps, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 4, L.OPT_GRAPH: 1})
    sim.step(8)
    sim.set_tool(0, 0, probe)
    sim.step(8)
    o = oracle_sim_like(orc, sc_caps).run(8)
    o2 = oracle_sim_like(orc, sc)
    o2.state = o.state
    o2.run(8)
    err = np.abs(sim.particles()[0] - o2.state.x).max()
    _say(f"  max |dx| = {err:.2e}")
    assert err <= TOL_DRIFT


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("kind,interp", KINDS, ids=KIND_IDS)
def test_adjoint_tools_match_oracle(gpu, orc, kind, interp):
    Sim, L, torch = gpu
    S, N, n, k = 10, 2000, 32, 4
    _say(f"adjoint vs oracle adjoint: {kind} interp={interp}, {N} particles, {n}^3, {S} substeps, checkpoints every {k}")
    sc = _scene(kind, interp, N=N, n=n, S=S, seed=71, perturb=True)
    env = sc.envs[0]
    rng = np.random.default_rng(72)
    for t in env.tools:
        t.traj = (t.traj[0] + 0.05 * rng.standard_normal((S, 3))).astype(np.float32)
    W = [rng.standard_normal((N, 3)), rng.standard_normal((N, 3)), rng.standard_normal((N, 3, 3)),
         rng.standard_normal((N, 3, 3))]
    sim = Sim(sc, max_tape=S, checkpoint_every=k, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 3})
    sim.step(S, record_tape=True)
    soa = lambda a, c: torch.tensor(a.reshape(N, c).T.copy(), dtype=torch.float32)
    g = sim.adjoint(S, soa(W[0], 3), soa(W[1], 3), soa(W[2], 9), soa(W[3], 9))
    o = oracle_sim_like(orc, sc).adjoint(S, *W)
    assert np.abs(o["gu"]).max() > 0
    nt = len(env.tools)
    checks = {
        "xbar0": (g["xbar0"].cpu().numpy().T, o["xbar"].reshape(N, 3)),
        "Fbar0": (g["Fbar0"].cpu().numpy().T, o["Fbar"].reshape(N, 9)),
        "gE": (g["gE"].cpu().numpy(), [o["gE"]]),
        "gnu": (g["gnu"].cpu().numpy(), [o["gnu"]]),
    }
    for t in range(nt):
        checks[f"gu{t}"] = (g["gu"].cpu().numpy()[0, t], o["gu"][:, t])
        checks[f"gT{t}"] = (g["gT"].cpu().numpy()[0, t], o["gT0"][t])
    for name, (a, b) in checks.items():
        e = _rel(a, b)
        _say(f"  {name}: rel err {e:.2e}")
        assert e <= 1e-3, (name, e)


def test_tool_argument_errors(gpu):
    Sim, L, torch = gpu
    _say("mpm_set_tool argument checks")
    sc = _scene("gripper", scenes.SDF_TRILINEAR, N=500, S=2)
    sim = Sim(sc)
    u = torch.zeros((1, 3), dtype=torch.float32, device="cuda")
    S = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")

    def call(**kw):
        base = dict(shape=L.TOOL_BOX, contact=0, radius=0.0, half_len=0.0, friction=0.3, theta=1e-3,
                    R=(ct.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1), T0=(ct.c_float * 3)(0.5, 0.5, 0.5),
                    half=(ct.c_float * 3)(0.01, 0.01, 0.01))
        base.update(kw)
        td = L.MpmTool(**base)
        return sim.lib.mpm_set_tool(sim.ctx, 0, 0, ct.byref(td), ct.c_void_p(u.data_ptr()), 1)

    assert call() == 0
    assert call(half=(ct.c_float * 3)(0.01, -0.01, 0.01)) == L.MPM_E_ARG
    assert call(radius=-1.0) == L.MPM_E_ARG
    assert call(shape=7) == L.MPM_E_ARG
    assert call(shape=L.TOOL_SDF) == L.MPM_E_ARG                       # no samples
    sdf = dict(shape=L.TOOL_SDF, sdf=S.data_ptr(), sdf_res=8, sdf_h=0.01, sdf_interp=L.SDF_TRILINEAR)
    assert call(**sdf) == 0
    assert call(**{**sdf, "sdf_res": 3}) == L.MPM_E_ARG
    assert call(**{**sdf, "sdf_h": 0.0}) == L.MPM_E_ARG
    assert call(**{**sdf, "sdf_interp": 2}) == L.MPM_E_ARG
    assert call(**{**sdf, "sdf_lo": (ct.c_float * 3)(0, float("nan"), 0)}) == L.MPM_E_ARG
    assert call(shape=L.TOOL_CAPSULE, radius=0.0) == L.MPM_E_ARG
    sim.close()
