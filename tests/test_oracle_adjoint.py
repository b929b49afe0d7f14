"""The oracle's hand adjoint against FP64 central finite differences of the
oracle's forward substeps (gradients of a random linear functional of the
final state with respect to E, nu, the per-substep tool velocities, the
initial tool pose and the initial particle state)."""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes


def _scene(seed, N, n, S, contact=scenes.CONTACT_SLIP, u=(0.05, -0.4, 0.02), friction=0.3, perturb=True):
    sc = scenes.small_slab_scene(seed, N, n=n, substeps=S, contact=contact, u=u, friction=friction, dt=1e-4)
    env = sc.envs[0]
    rng = np.random.default_rng(seed + 7)
    if perturb:
        scenes.perturbed_state(rng, env, v_scale=0.05, C_scale=1.0, F_scale=0.01)
    # per-substep velocities with some variation so each entry matters
    base = np.asarray(u, np.float64)
    env.tools[0].traj = (base + 0.05 * rng.standard_normal((S, 3))).astype(np.float32)
    # lower the tool a bit so a band of nodes is in contact from the start
    env.tools[0].T0 = (env.tools[0].T0 - np.array([0, 0.015, 0])).astype(np.float32)
    return sc, env


def _functional(seed, N):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((N, 3)), rng.standard_normal((N, 3)),
            rng.standard_normal((N, 3, 3)), rng.standard_normal((N, 3, 3)))


def _L(sim, W):
    st = sim.state
    return sum((a * b).sum() for a, b in zip((st.x, st.v, st.C, st.F), W))


def _run(orc, sc, env, S, E=None, nu=None, traj=None, T0=None, state=None):
    sim = orc.Sim(env, dt=sc.dt, E=E, nu=nu)
    if traj is not None:
        sim.traj[0] = traj
    if T0 is not None:
        sim.T[0] = T0
    if state is not None:
        sim.state = state
    sim.run(S)
    return sim


@pytest.mark.parametrize("contact", [scenes.CONTACT_SLIP, scenes.CONTACT_STICKY])
def test_adjoint_vs_fd(orc, contact):
    S, N, n = 6, 300, 32
    sc, env = _scene(31 + contact, N, n, S, contact=contact)
    W = _functional(5, N)
    sim = orc.Sim(env, dt=sc.dt)
    g = sim.adjoint(S, *W)
    assert g["flags"] == 0
    # the tool touches nodes, so its gradients are not trivially zero
    assert np.abs(g["gu"]).max() > 0

    # E and nu
    for key, val, h in (("gE", env.E, 1e-3), ("gnu", env.nu, 1e-7)):
        kw = lambda d: {("E" if key == "gE" else "nu"): val + d}
        fd = (_L(_run(orc, sc, env, S, **kw(h)), W) - _L(_run(orc, sc, env, S, **kw(-h)), W)) / (2 * h)
        assert g[key] == pytest.approx(fd, rel=2e-6, abs=1e-9 * abs(fd) + 1e-12), key

    # per-substep tool velocity, a few entries
    traj0 = sim.traj[0].copy()
    rng = np.random.default_rng(1)
    for s, a in [(0, 1), (S // 2, 0), (S - 1, 2), (1, 1)]:
        h = 1e-6
        tp, tm = traj0.copy(), traj0.copy()
        tp[s, a] += h
        tm[s, a] -= h
        fd = (_L(_run(orc, sc, env, S, traj=tp), W) - _L(_run(orc, sc, env, S, traj=tm), W)) / (2 * h)
        assert g["gu"][s, 0, a] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g["gu"]).max()), (s, a)

    # initial tool pose
    for a in range(3):
        h = 1e-7
        T0 = np.asarray(env.tools[0].T0, np.float64)
        Tp, Tm = T0.copy(), T0.copy()
        Tp[a] += h
        Tm[a] -= h
        fd = (_L(_run(orc, sc, env, S, T0=Tp), W) - _L(_run(orc, sc, env, S, T0=Tm), W)) / (2 * h)
        assert g["gT0"][0, a] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g["gT0"]).max() + 1e-9), a

    # initial particle state, random directions
    st0 = orc.State.from_env(env)
    for field, h in (("x", 1e-8), ("v", 1e-6), ("C", 1e-5), ("F", 1e-7)):
        d = rng.standard_normal(getattr(st0, field).shape)
        sp, sm = st0.copy(), st0.copy()
        setattr(sp, field, getattr(sp, field) + h * d)
        setattr(sm, field, getattr(sm, field) - h * d)
        fd = (_L(_run(orc, sc, env, S, state=sp), W) - _L(_run(orc, sc, env, S, state=sm), W)) / (2 * h)
        an = (g[field + "bar"] * d).sum()
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-7 * abs(fd) + 1e-10), field


def test_adjoint_friction_branch_dominant(orc):
    """Large tangential motion under the tool so most contact nodes take the
    friction branch (not the clamp)."""
    S, N, n = 4, 250, 32
    sc, env = _scene(41, N, n, S, u=(0.6, -0.3, 0.0), friction=0.2)
    env.v[:, 0] = -0.8
    W = _functional(9, N)
    sim = orc.Sim(env, dt=sc.dt)
    g = sim.adjoint(S, *W)
    traj0 = sim.traj[0].copy()
    for s, a in [(0, 0), (2, 1), (3, 0)]:
        h = 1e-6
        tp, tm = traj0.copy(), traj0.copy()
        tp[s, a] += h
        tm[s, a] -= h
        fd = (_L(_run(orc, sc, env, S, traj=tp), W) - _L(_run(orc, sc, env, S, traj=tm), W)) / (2 * h)
        assert g["gu"][s, 0, a] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g["gu"]).max())
    # friction branch nodes exist in the first substep
    gm, gmv = sim.p2g()
    gv, rec = sim.grid_update(gm, gmv, record=True)
    branches = np.array([r.branch for r in rec])
    assert (branches == 1).sum() > 0


def test_adjoint_no_tool_matches_fd(orc):
    """Config-1-like cube, no tool, more substeps."""
    sc = scenes.cube_scene(substeps=8)
    env = sc.envs[0]
    keep = np.random.default_rng(3).choice(env.N, 400, replace=False)
    env.x, env.v, env.C, env.F = env.x[keep], env.v[keep], env.C[keep], env.F[keep]
    scenes.perturbed_state(np.random.default_rng(4), env, v_scale=0.1, C_scale=1.0, F_scale=0.01)
    S = sc.substeps
    W = _functional(2, env.N)
    g = orc.Sim(env, dt=sc.dt).adjoint(S, *W)
    for key, val, h in (("gE", env.E, 1e-3), ("gnu", env.nu, 1e-7)):
        kw = lambda d: {("E" if key == "gE" else "nu"): val + d}
        fd = (_L(_run(orc, sc, env, S, **kw(h)), W) - _L(_run(orc, sc, env, S, **kw(-h)), W)) / (2 * h)
        assert g[key] == pytest.approx(fd, rel=2e-6), key
