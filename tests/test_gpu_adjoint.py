"""The GPU adjoint (mpm_substep_adjoint through the C ABI and the autograd
Function) against the FP64 oracle's adjoint and FP64 central finite
differences of the oracle.  Gradients are held to 1e-3 relative."""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes
from parity import oracle_sim_like

pytestmark = pytest.mark.gpu
TOL_GRAD = 1e-3


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


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def _pressing_scene(seed, N, n, S, contact=scenes.CONTACT_SLIP):
    sc = scenes.small_slab_scene(seed, N, n=n, substeps=S, contact=contact, u=(0.05, -0.4, 0.02), dt=1e-4)
    env = sc.envs[0]
    rng = np.random.default_rng(seed + 1)
    scenes.perturbed_state(rng, env, v_scale=0.05, C_scale=1.0, F_scale=0.01)
    env.tools[0].traj = (np.array([0.05, -0.4, 0.02]) + 0.05 * rng.standard_normal((S, 3))).astype(np.float32)
    env.tools[0].T0 = (env.tools[0].T0 - np.array([0, 0.015, 0])).astype(np.float32)
    return sc, env


@pytest.mark.parametrize("scheme,contact,slots,pers", [("tiled", scenes.CONTACT_SLIP, 3, 0),
                                                       ("direct", scenes.CONTACT_SLIP, 3, 0),
                                                       ("tiled", scenes.CONTACT_STICKY, 3, 0),
                                                       ("tiled", scenes.CONTACT_SLIP, 1, 0),
                                                       ("tiled", scenes.CONTACT_SLIP, 3, 1),
                                                       ("tiled", scenes.CONTACT_STICKY, 1, 1)])
def test_adjoint_matches_oracle_adjoint(gpu, orc, scheme, contact, slots, pers):
    """Every gradient against the oracle's FP64 adjoint; pers: the recorded
    forward takes persistent runs of the grid at staging."""
    Sim, L, torch = gpu
    S, N, n, k = 12, 2000, 32, 5
    _say(f"adjoint vs oracle adjoint: {N} particles, {n}^3, {S} substeps, checkpoints every {k}, {scheme}, "
         f"contact={contact}, node slots {slots}, persistent {pers}")
    sc, env = _pressing_scene(51 + contact, N, n, S, contact)
    rng = np.random.default_rng(3)
    W = [rng.standard_normal((N, 3)), rng.standard_normal((N, 3)), rng.standard_normal((N, 3, 3)),
         rng.standard_normal((N, 3, 3))]
    sim = Sim(sc, max_tape=S, checkpoint_every=k,
              options={L.OPT_SCHEME: L.SCHEME_TILED if scheme == "tiled" else L.SCHEME_DIRECT, L.OPT_SORT_EVERY: 3,
                       L.OPT_NODE_SLOTS: slots, L.OPT_PERSISTENT: pers, L.OPT_GRID_AT_STAGING: pers})
    sim.step(S, record_tape=True)
    soa = lambda a, c: torch.tensor(a.reshape(N, c).T.copy(), dtype=torch.float32)
    g = sim.adjoint(S, soa(W[0], 3), soa(W[1], 3), soa(W[2], 9), soa(W[3], 9))
    o = oracle_sim_like(orc, sc).adjoint(S, *W)
    assert np.abs(o["gu"]).max() > 0
    checks = {
        "xbar0": (g["xbar0"].cpu().numpy().T, o["xbar"].reshape(N, 3)),
        "vbar0": (g["vbar0"].cpu().numpy().T, o["vbar"].reshape(N, 3)),
        "Cbar0": (g["Cbar0"].cpu().numpy().T, o["Cbar"].reshape(N, 9)),
        "Fbar0": (g["Fbar0"].cpu().numpy().T, o["Fbar"].reshape(N, 9)),
        "gE": (g["gE"].cpu().numpy(), [o["gE"]]),
        "gnu": (g["gnu"].cpu().numpy(), [o["gnu"]]),
        "gu": (g["gu"].cpu().numpy()[0, 0], o["gu"][:, 0]),
        "gT": (g["gT"].cpu().numpy()[0, 0], o["gT0"][0]),
    }
    for name, (a, b) in checks.items():
        e = _rel(a, b)
        _say(f"  {name}: rel err {e:.2e}")
        assert e <= TOL_GRAD, (name, e)


def test_held_tape_matches_oracle_adjoint(gpu, orc):
    """A recording kept whole (hold_tape): the forward runs the recompute
    passes segment by segment (three segments, the last one short) and the
    adjoint reverses the held tapes without recomputing.  Every gradient
    against the oracle's FP64 adjoint; the final forward state against the
    ordinary forward's; a second adjoint of the same recording (the held
    tapes are consumed, so it recomputes from the checkpoints) and a reverse
    window shorter than the recording against the oracle too."""
    Sim, L, torch = gpu
    S, N, n, k = 12, 2000, 32, 5
    _say(f"held tape: {N} particles, {n}^3, {S} substeps, segments of {k}")
    sc, env = _pressing_scene(53, N, n, S)
    rng = np.random.default_rng(8)
    W = [rng.standard_normal((N, 3)), rng.standard_normal((N, 3)), rng.standard_normal((N, 3, 3)),
         rng.standard_normal((N, 3, 3))]
    opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 3}
    soa = lambda a, c: torch.tensor(a.reshape(N, c).T.copy(), dtype=torch.float32)
    plain = Sim(sc, max_tape=S, checkpoint_every=k, options=opts)
    plain.step(S, record_tape=True)
    held = Sim(sc, max_tape=S, checkpoint_every=k, options=opts, hold_tape=True)
    assert held.workspace_bytes > plain.workspace_bytes
    held.step(S, record_tape=True)
    for a, b, name in zip(held.particles(), plain.particles(), ("x", "v", "C", "F")):
        e = _rel(a, b)
        _say(f"  final {name}: held vs ordinary forward rel err {e:.2e}")
        assert e <= 1e-4, (name, e)
    np.testing.assert_array_equal(held.read(L.F_TOOL_T), plain.read(L.F_TOOL_T))
    o = oracle_sim_like(orc, sc).adjoint(S, *W)

    def check(g, what):
        checks = {
            "xbar0": (g["xbar0"].cpu().numpy().T, o["xbar"].reshape(N, 3)),
            "vbar0": (g["vbar0"].cpu().numpy().T, o["vbar"].reshape(N, 3)),
            "Cbar0": (g["Cbar0"].cpu().numpy().T, o["Cbar"].reshape(N, 9)),
            "Fbar0": (g["Fbar0"].cpu().numpy().T, o["Fbar"].reshape(N, 9)),
            "gE": (g["gE"].cpu().numpy(), [o["gE"]]),
            "gnu": (g["gnu"].cpu().numpy(), [o["gnu"]]),
            "gu": (g["gu"].cpu().numpy()[0, 0], o["gu"][:, 0]),
            "gT": (g["gT"].cpu().numpy()[0, 0], o["gT0"][0]),
        }
        for name, (a, b) in checks.items():
            e = _rel(a, b)
            _say(f"  {what} {name}: rel err {e:.2e}")
            assert e <= TOL_GRAD, (what, name, e)

    seeds = (soa(W[0], 3), soa(W[1], 3), soa(W[2], 9), soa(W[3], 9))
    check(held.adjoint(S, *seeds), "held")
    check(held.adjoint(S, *seeds), "recomputed")
    # a reverse window of 7 of the 12 recorded substeps
    held.close()
    held = Sim(sc, max_tape=S, checkpoint_every=k, options=opts, hold_tape=True)
    held.step(S, record_tape=True)
    w = 7
    gw = held.adjoint(w, seeds[0])
    plain_w = plain.adjoint(w, seeds[0])
    for name in ("xbar0", "vbar0", "Cbar0", "Fbar0", "gE", "gnu", "gu", "gT"):
        e = _rel(gw[name].cpu().numpy(), plain_w[name].cpu().numpy())
        _say(f"  window {w}: {name} held vs recomputed rel err {e:.2e}")
        assert e <= TOL_GRAD, (name, e)
    held.close()
    plain.close()


@pytest.mark.parametrize("pers", [0, 1])
def test_adjoint_with_particles_leaving_their_tiles(gpu, orc, pers):
    """The slab and the tool translate at 80 m/s along x, so within one tape
    segment (6 substeps, one sort at its start) every particle moves more than
    a cell and those at brick edges leave their work item's tile: the reverse
    G2P and P2G passes then read node values from the global grid instead of
    the LDS tile.  Gradients against the oracle's adjoint."""
    Sim, L, torch = gpu
    S, N, n, k = 12, 2000, 32, 6
    drift = np.array([80.0, 0.0, 0.0])
    sc, env = _pressing_scene(71, N, n, S)
    env.v = (env.v + drift).astype(np.float32)
    env.tools[0].traj = (env.tools[0].traj + drift).astype(np.float32)
    _say(f"adjoint with tile drift: {N} particles, {n}^3, {S} substeps, checkpoints every {k}, drift {drift[0]} m/s")
    o_fwd = oracle_sim_like(orc, sc)
    x0 = o_fwd.state.x.copy()
    o_fwd.run(k)
    moved = (o_fwd.state.x[:, 0] - x0[:, 0]) * n   # in cells
    _say(f"  displacement over one segment: {moved.min():.2f}..{moved.max():.2f} cells")
    assert moved.min() > 1.0
    rng = np.random.default_rng(5)
    W = [rng.standard_normal((N, 3)), rng.standard_normal((N, 3)), rng.standard_normal((N, 3, 3)),
         rng.standard_normal((N, 3, 3))]
    sim = Sim(sc, max_tape=S, checkpoint_every=k,
              options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: k, L.OPT_PERSISTENT: pers})
    sim.step(S, record_tape=True)
    assert sim.read(L.F_STATUS) == 0
    soa = lambda a, c: torch.tensor(a.reshape(N, c).T.copy(), dtype=torch.float32)
    g = sim.adjoint(S, soa(W[0], 3), soa(W[1], 3), soa(W[2], 9), soa(W[3], 9))
    o = oracle_sim_like(orc, sc).adjoint(S, *W)
    assert np.abs(o["gu"]).max() > 0
    checks = {
        "xbar0": (g["xbar0"].cpu().numpy().T, o["xbar"].reshape(N, 3)),
        "vbar0": (g["vbar0"].cpu().numpy().T, o["vbar"].reshape(N, 3)),
        "Cbar0": (g["Cbar0"].cpu().numpy().T, o["Cbar"].reshape(N, 9)),
        "Fbar0": (g["Fbar0"].cpu().numpy().T, o["Fbar"].reshape(N, 9)),
        "gE": (g["gE"].cpu().numpy(), [o["gE"]]),
        "gnu": (g["gnu"].cpu().numpy(), [o["gnu"]]),
        "gu": (g["gu"].cpu().numpy()[0, 0], o["gu"][:, 0]),
    }
    for name, (a, b) in checks.items():
        e = _rel(a, b)
        _say(f"  {name}: rel err {e:.2e}")
        assert e <= TOL_GRAD, (name, e)


def test_held_tape_grids_cleared_before_reuse(gpu, orc):
    """Tape grids of a held recording that no reverse pass cleared: a reverse
    window shorter than the recording leaves the earlier segments' grids, and
    a recording made over one that was never reversed finds all of them.  A
    recompute into such a segment must start from zero grids: the whole
    adjoint after a window of 7 (its first segment recomputed), and a second
    held recording (its forward state and its adjoint), against the oracle.
    The tool velocity is constant, so the second recording's substeps take
    the same trajectory entries on both sides."""
    Sim, L, torch = gpu
    S, N, n, k = 12, 2000, 32, 5
    sc, env = _pressing_scene(54, N, n, 2 * S)
    env.tools[0].traj = np.tile(env.tools[0].traj[0], (2 * S, 1)).astype(np.float32)
    _say(f"held tape reuse: {N} particles, {n}^3, {S} substeps, segments of {k}")
    rng = np.random.default_rng(11)
    W = [rng.standard_normal((N, 3)), rng.standard_normal((N, 3)), rng.standard_normal((N, 3, 3)),
         rng.standard_normal((N, 3, 3))]
    opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 3}
    soa = lambda a, c: torch.tensor(a.reshape(N, c).T.copy(), dtype=torch.float32)
    seeds = (soa(W[0], 3), soa(W[1], 3), soa(W[2], 9), soa(W[3], 9))

    def check(g, o, what):
        assert np.abs(o["gu"]).max() > 0
        checks = {
            "xbar0": (g["xbar0"].cpu().numpy().T, o["xbar"].reshape(N, 3)),
            "vbar0": (g["vbar0"].cpu().numpy().T, o["vbar"].reshape(N, 3)),
            "Cbar0": (g["Cbar0"].cpu().numpy().T, o["Cbar"].reshape(N, 9)),
            "Fbar0": (g["Fbar0"].cpu().numpy().T, o["Fbar"].reshape(N, 9)),
            "gE": (g["gE"].cpu().numpy(), [o["gE"]]),
            "gnu": (g["gnu"].cpu().numpy(), [o["gnu"]]),
            "gu": (g["gu"].cpu().numpy()[0, 0], o["gu"][:, 0]),
            "gT": (g["gT"].cpu().numpy()[0, 0], o["gT0"][0]),
        }
        for name, (a, b) in checks.items():
            e = _rel(a, b)
            _say(f"  {what} {name}: rel err {e:.2e}")
            assert e <= TOL_GRAD, (what, name, e)

    held = Sim(sc, max_tape=S, checkpoint_every=k, options=opts, hold_tape=True)
    held.step(S, record_tape=True)
    held.adjoint(7, seeds[0])
    check(held.adjoint(S, *seeds), oracle_sim_like(orc, sc).adjoint(S, *W), "whole after a window of 7")
    held.close()

    held = Sim(sc, max_tape=S, checkpoint_every=k, options=opts, hold_tape=True)
    held.step(S, record_tape=True)
    held.step(S, record_tape=True)
    o = oracle_sim_like(orc, sc)
    o.run(S)
    o.run(S)
    x = held.read(L.F_X).cpu().numpy().T
    e = float(np.abs(x - o.state.x).max())
    _say(f"  second recording: final positions vs oracle max |dx| {e:.2e} m")
    # FP32 against FP64 over 24 substeps stays near 5e-7 m here; stale grids shift
    # the velocities the forward itself integrates
    assert e <= 5e-6, e
    o = oracle_sim_like(orc, sc)
    o.run(S)
    check(held.adjoint(S, *seeds), o.adjoint(S, *W), "second recording")
    held.close()


def test_held_tape_option_with_direct_scheme(gpu, orc):
    """hold_tape with the direct (untiled) scheme: the recording keeps
    checkpoints only and every adjoint recomputes, each segment into its own
    tape buffers.  Two adjoints of one recording against the oracle."""
    Sim, L, torch = gpu
    S, N, n, k = 12, 2000, 32, 5
    sc, env = _pressing_scene(55, N, n, S)
    _say(f"held tape option, direct scheme: {N} particles, {n}^3, {S} substeps, segments of {k}")
    rng = np.random.default_rng(12)
    W = [rng.standard_normal((N, 3)), rng.standard_normal((N, 3)), rng.standard_normal((N, 3, 3)),
         rng.standard_normal((N, 3, 3))]
    soa = lambda a, c: torch.tensor(a.reshape(N, c).T.copy(), dtype=torch.float32)
    seeds = (soa(W[0], 3), soa(W[1], 3), soa(W[2], 9), soa(W[3], 9))
    sim = Sim(sc, max_tape=S, checkpoint_every=k, options={L.OPT_SCHEME: L.SCHEME_DIRECT}, hold_tape=True)
    sim.step(S, record_tape=True)
    o = oracle_sim_like(orc, sc).adjoint(S, *W)
    for what in ("first", "second"):
        g = sim.adjoint(S, *seeds)
        checks = {
            "xbar0": (g["xbar0"].cpu().numpy().T, o["xbar"].reshape(N, 3)),
            "Fbar0": (g["Fbar0"].cpu().numpy().T, o["Fbar"].reshape(N, 9)),
            "gE": (g["gE"].cpu().numpy(), [o["gE"]]),
            "gu": (g["gu"].cpu().numpy()[0, 0], o["gu"][:, 0]),
            "gT": (g["gT"].cpu().numpy()[0, 0], o["gT0"][0]),
        }
        for name, (a, b) in checks.items():
            e = _rel(a, b)
            _say(f"  {what} adjoint {name}: rel err {e:.2e}")
            assert e <= TOL_GRAD, (what, name, e)
    sim.close()


@pytest.mark.parametrize("pers,hold", [(0, False), (1, True)])
def test_adjoint_two_environments_match_oracle(gpu, orc, pers, hold):
    """Two environments of different sizes (32^3 and 64^3 grids), particle
    counts, materials and tool paths in one context: the reverse grid passes
    then look up each brick's environment and tool slots, and the gradient
    chain runs once per (environment, tool).  Each environment's gradients
    against the oracle's adjoint of that environment alone; hold: the tape
    kept whole."""
    Sim, L, torch = gpu
    S, k = 12, 5
    sa, ea = _pressing_scene(81, 1500, 32, S)
    sb, eb = _pressing_scene(82, 2500, 64, S, scenes.CONTACT_STICKY)
    eb.E, eb.nu = float(np.float32(2.5e4)), float(np.float32(0.3))
    sc = scenes.Scene("two-slabs", [ea, eb], dt=sa.dt, substeps=S)
    sizes = [ea.x.shape[0], eb.x.shape[0]]
    ofs = np.concatenate([[0], np.cumsum(sizes)])
    _say(f"adjoint, two environments: {sizes} particles on 32^3 / 64^3, {S} substeps, checkpoints every {k}, "
         f"persistent {pers}, held tape {hold}")
    rng = np.random.default_rng(9)
    W = [[rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), rng.standard_normal((n, 3, 3)),
          rng.standard_normal((n, 3, 3))] for n in sizes]
    sim = Sim(sc, max_tape=S, checkpoint_every=k, hold_tape=hold,
              options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_SORT_EVERY: 3, L.OPT_PERSISTENT: pers,
                       L.OPT_GRID_AT_STAGING: pers})
    sim.step(S, record_tape=True)
    assert [sim.read(L.F_STATUS, e) for e in range(2)] == [0, 0]
    soa = lambda f, c: torch.tensor(np.concatenate([w[f].reshape(-1, c) for w in W]).T.copy(), dtype=torch.float32)
    g = sim.adjoint(S, soa(0, 3), soa(1, 3), soa(2, 9), soa(3, 9))
    for e in range(2):
        o = oracle_sim_like(orc, sc, e).adjoint(S, *W[e])
        assert np.abs(o["gu"]).max() > 0
        sl = slice(int(ofs[e]), int(ofs[e + 1]))
        n = sizes[e]
        checks = {
            "xbar0": (g["xbar0"][:, sl].cpu().numpy().T, o["xbar"].reshape(n, 3)),
            "vbar0": (g["vbar0"][:, sl].cpu().numpy().T, o["vbar"].reshape(n, 3)),
            "Cbar0": (g["Cbar0"][:, sl].cpu().numpy().T, o["Cbar"].reshape(n, 9)),
            "Fbar0": (g["Fbar0"][:, sl].cpu().numpy().T, o["Fbar"].reshape(n, 9)),
            "gE": (g["gE"].cpu().numpy()[e:e + 1], [o["gE"]]),
            "gnu": (g["gnu"].cpu().numpy()[e:e + 1], [o["gnu"]]),
            "gu": (g["gu"].cpu().numpy()[e, 0], o["gu"][:, 0]),
            "gT": (g["gT"].cpu().numpy()[e, 0], o["gT0"][0]),
        }
        for name, (a, b) in checks.items():
            err = _rel(a, b)
            _say(f"  env {e} {name}: rel err {err:.2e}")
            assert err <= TOL_GRAD, (e, name, err)


@pytest.mark.parametrize("pers", [0, 1])
def test_adjoint_window_shorter_than_tape(gpu, orc, pers):
    """Reverse only the last 7 of 12 recorded substeps."""
    Sim, L, torch = gpu
    S, N, n, k, w = 12, 1500, 32, 4, 7
    _say(f"adjoint window {w} of {S} substeps, persistent {pers}")
    sc, env = _pressing_scene(61, N, n, S)
    rng = np.random.default_rng(4)
    Wx = rng.standard_normal((N, 3))
    sim = Sim(sc, max_tape=S, checkpoint_every=k, options={L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_PERSISTENT: pers})
    sim.step(S, record_tape=True)
    g = sim.adjoint(w, torch.tensor(Wx.T.copy(), dtype=torch.float32))
    o = oracle_sim_like(orc, sc)
    o.run(S - w)
    # the oracle adjoint restarts at substep S - w from its own FP64 state and tool pose
    o.traj = np.ascontiguousarray(o.traj[:, S - w:])
    o.n_traj = o.traj.shape[1]
    ref = o.adjoint(w, Wx)
    for name, a, b in (("xbar0", g["xbar0"].cpu().numpy().T, ref["xbar"]), ("gE", g["gE"].cpu().numpy(), [ref["gE"]]),
                       ("gu", g["gu"].cpu().numpy()[0, 0], ref["gu"][:, 0])):
        e = _rel(a, b)
        _say(f"  {name}: rel err {e:.2e}")
        assert e <= TOL_GRAD, (name, e)


@pytest.mark.parametrize("shipped", [0, 1])
def test_autograd_diff_slab_full_size_vs_fd(gpu, orc, shipped):
    """The differentiable workload at full size: 30K particles, 64^3, 200
    substeps, checkpoints every 20; loss = |centroid - target|^2; gradients
    with respect to E, nu and the 200 tool velocities against FP64 central
    differences of the oracle.  shipped: the slab's benchmark launch options
    (the forward in persistent runs of the grid at staging)."""
    Sim, L, torch = gpu
    from paper_2402_01181_amd.autograd import MPMRollout
    sc = scenes.diff_scene()
    env = sc.envs[0]
    S = sc.substeps
    target = torch.tensor(sc.extra["target"], dtype=torch.float64)
    opts = {}
    if shipped:
        opts = {L.OPT_SCHEME: L.SCHEME_TILED, L.OPT_BLOCK: 256, L.OPT_ITEM: 160, L.OPT_SORT_EVERY: 32,
                L.OPT_NODE_SLOTS: 3, L.OPT_GRID_AT_STAGING: 1, L.OPT_PERSISTENT: 1}
    _say(f"autograd rollout: {env.N} particles, {S} substeps, checkpoints every {sc.extra['checkpoint_every']}, "
         f"options {opts}")
    sim = Sim(sc, max_tape=S, checkpoint_every=sc.extra["checkpoint_every"], options=opts)
    E = torch.tensor([env.E], dtype=torch.float64, requires_grad=True)
    nu = torch.tensor([env.nu], dtype=torch.float64, requires_grad=True)
    u = torch.tensor(env.tools[0].traj[None, None], dtype=torch.float64, requires_grad=True)
    x, v = MPMRollout.apply(E, nu, u, sim, S)
    loss = ((x.double().mean(0).cpu() - target) ** 2).sum()
    loss.backward()
    assert sim.read(L.F_STATUS) == 0

    def oracle_loss(E_=None, nu_=None, traj=None):
        o = oracle_sim_like(orc, sc)
        if E_ is not None:
            o.P.E = E_
        if nu_ is not None:
            o.P.nu = nu_
        if traj is not None:
            o.traj[0] = traj
        o.run(S)
        c = o.state.x.mean(0)
        return float(((c - sc.extra["target"]) ** 2).sum())

    L0 = oracle_loss()
    _say(f"  loss gpu {loss.item():.6e} oracle {L0:.6e}")
    assert abs(loss.item() - L0) <= 1e-3 * L0
    # the oracle's own FP64 adjoint of the same loss
    o = oracle_sim_like(orc, sc)
    c0 = None
    ref = None
    oo = oracle_sim_like(orc, sc).run(S)
    c0 = oo.state.x.mean(0)
    xbar = np.tile(2.0 * (c0 - sc.extra["target"]) / env.N, (env.N, 1))
    ref = o.adjoint(S, xbar)
    for name, a, b in (("dL/dE", E.grad.item(), ref["gE"]), ("dL/dnu", nu.grad.item(), ref["gnu"]),
                       ("dL/du", u.grad[0, 0].numpy(), ref["gu"][:, 0])):
        e = _rel(a, b)
        _say(f"  {name} vs oracle adjoint: rel {e:.2e}")
        assert e <= TOL_GRAD, (name, e)
    hE, hnu = 1e-3 * env.E, 1e-5
    fdE = (oracle_loss(E_=env.E + hE) - oracle_loss(E_=env.E - hE)) / (2 * hE)
    fdnu = (oracle_loss(nu_=env.nu + hnu) - oracle_loss(nu_=env.nu - hnu)) / (2 * hnu)
    rng = np.random.default_rng(11)
    d = rng.standard_normal((S, 3))
    hu = 1e-6   # small: the tool path moves < 1e-8 m, so no contact decision changes
    traj0 = env.tools[0].traj.astype(np.float64)
    fdu = (oracle_loss(traj=traj0 + hu * d) - oracle_loss(traj=traj0 - hu * d)) / (2 * hu)
    gu_dir = float((u.grad[0, 0].numpy() * d).sum())
    for name, a, b in (("dL/dE", E.grad.item(), fdE), ("dL/dnu", nu.grad.item(), fdnu), ("dL/du . d", gu_dir, fdu)):
        e = abs(a - b) / max(abs(b), 1e-30)
        _say(f"  {name}: adjoint {a:.6e} fd {b:.6e} rel {e:.2e}")
        assert e <= TOL_GRAD, (name, a, b)


def test_adjoint_state_errors(gpu, orc):
    Sim, L, torch = gpu
    sc = scenes.small_slab_scene(5, 300, n=16, substeps=4)
    sim = Sim(sc, max_tape=4, checkpoint_every=2)
    with pytest.raises(L.MpmError) as ei:
        sim.adjoint(2)
    assert ei.value.code == L.MPM_E_STATE
    with pytest.raises(L.MpmError) as ei:
        sim.step(5, record_tape=True)
    assert ei.value.code == L.MPM_E_ARG
    sim.step(3, record_tape=True)
    with pytest.raises(L.MpmError) as ei:
        sim.adjoint(4)
    assert ei.value.code == L.MPM_E_STATE
    sim.adjoint(3)
    sim.step(1)                        # stepping on invalidates the tape
    with pytest.raises(L.MpmError) as ei:
        sim.adjoint(1)
    assert ei.value.code == L.MPM_E_STATE
    nt = Sim(sc)                       # no tape capacity
    with pytest.raises(L.MpmError) as ei:
        nt.step(1, record_tape=True)
    assert ei.value.code == L.MPM_E_STATE
