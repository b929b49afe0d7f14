"""Pins of the oracle's box and sampled-SDF tools (Sec. III-C: bounding boxes
for the gripper jaws, a precomputed SDF indexed in the tool frame with
central-difference normals, the z-buffer over several tools).

Each check is against something other than the oracle itself: distances by
brute force over sampled surfaces, gradients by finite differences, exact
reproduction of linear fields by trilinear interpolation, the paper's
integer indexing, the capsule as a degenerate rounded box, and the adjoint
against finite differences of the forward substeps.
"""
import numpy as np
import pytest

from paper_2402_01181_amd import scenes


def _box_surface(half, m=160):
    """Points on the surface of the box [-half, half] (m x m per face)."""
    pts = []
    for a in range(3):
        b, c = [d for d in range(3) if d != a]
        u = np.linspace(-half[b], half[b], m)
        v = np.linspace(-half[c], half[c], m)
        U, V = np.meshgrid(u, v, indexing="ij")
        for sgn in (-1.0, 1.0):
            p = np.zeros((m * m, 3))
            p[:, a] = sgn * half[a]
            p[:, b] = U.ravel()
            p[:, c] = V.ravel()
            pts.append(p)
    return np.concatenate(pts)


def test_box_sdf_brute_force(orc):
    rng = np.random.default_rng(11)
    for _ in range(6):
        half = rng.uniform(0.005, 0.05, 3)
        surf = _box_surface(half)
        spacing = 2 * half.max() / 159
        for _ in range(25):
            p = rng.uniform(-2, 2, 3) * half
            d = np.linalg.norm(surf - p, axis=1).min()
            inside = np.all(np.abs(p) <= half)
            ref = -d if inside else d
            for r in (0.0, 0.004):
                phi, l, J = orc.box_sdf(p, half, r)
                assert phi == pytest.approx(ref - r, abs=spacing), (p, half)
                assert (phi + r < 0) == inside


def test_box_normal_and_jacobian_are_derivatives(orc):
    rng = np.random.default_rng(12)
    half = np.array([0.04, 0.01, 0.02])
    e = 1e-7
    n_in = n_out = 0
    for _ in range(300):
        p = rng.uniform(-2, 2, 3) * half
        a_ = np.abs(p) - half
        inside = np.all(a_ <= 0)
        # stay away from the medial planes inside and the clamp switches outside
        if inside and np.sort(a_)[-1] - np.sort(a_)[-2] < 1e-4:
            continue
        if np.min(np.abs(a_)) < 1e-4:
            continue
        phi, l, J = orc.box_sdf(p, half, 0.0)
        grad = np.array([(orc.box_sdf(p + e * np.eye(3)[k], half)[0] - orc.box_sdf(p - e * np.eye(3)[k], half)[0]) / (2 * e)
                         for k in range(3)])
        np.testing.assert_allclose(l, grad, atol=1e-6)
        assert np.linalg.norm(l) == pytest.approx(1.0, abs=1e-12)
        Jfd = np.stack([(orc.box_sdf(p + e * np.eye(3)[k], half)[1] - orc.box_sdf(p - e * np.eye(3)[k], half)[1]) / (2 * e)
                        for k in range(3)], 1)
        np.testing.assert_allclose(J, Jfd, atol=1e-4 * max(1.0, np.abs(Jfd).max()))
        n_in += inside
        n_out += not inside
    assert n_in > 10 and n_out > 10


def test_capsule_is_a_rounded_degenerate_box(orc):
    """A box with half extents (h, 0, 0) rounded by r is the capsule."""
    rng = np.random.default_rng(13)
    r, h = 0.02, 0.1
    for _ in range(200):
        p = rng.uniform(-0.2, 0.2, 3)
        phi_c, q, _ = orc.capsule_sdf(p, r, h)
        phi_b, l, _ = orc.box_sdf(p, [h, 0.0, 0.0], r)
        assert phi_b == pytest.approx(phi_c, abs=1e-15)
        np.testing.assert_allclose(l, q / np.linalg.norm(q), atol=1e-14)


def _linear_tool(a, c, res, h, lo, interp):
    ax = [lo[k] + h * np.arange(res) for k in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    S = a[0] * X + a[1] * Y + a[2] * Z - c
    return scenes.sdf_tool((0, 0, 0), S, h, lo, interp=interp)


def test_trilinear_reproduces_a_linear_field(orc):
    """Trilinear interpolation and central differences are exact on a plane:
    phi = a.x - c and l = a everywhere in the field, with dl/dx = 0."""
    rng = np.random.default_rng(14)
    res, h, lo = 24, 1.0 / 64, (-0.2, -0.1, -0.15)
    for _ in range(5):
        a = rng.standard_normal(3)
        a /= np.linalg.norm(a)
        c = rng.uniform(-0.05, 0.05)
        tool = _linear_tool(a, c, res, h, lo, scenes.SDF_TRILINEAR)
        lo32, h32 = np.asarray(tool.sdf_lo, np.float64), float(tool.sdf_h)
        for _ in range(40):
            s = rng.uniform(1.0, res - 2.0, 3)
            x = lo32 + s * h32
            phi, l, J = orc.sampled_sdf(tool, x)
            # only the f32 rounding of the samples separates it from the plane
            assert phi == pytest.approx(a @ x - c, abs=2e-7)
            np.testing.assert_allclose(l, a, atol=3e-5)
            assert np.abs(J).max() < 1e-2


def test_nearest_is_the_papers_index(orc):
    """Paper setting: lattice origin at the tool origin, spacing 1/256; the
    distance is SDF[x_ref/dx] with the index truncated and the normal is
    the central difference there."""
    rng = np.random.default_rng(15)
    res, h = 256, 1.0 / 256
    S = rng.standard_normal((res, res, res)).astype(np.float32)
    tool = scenes.sdf_tool((0, 0, 0), S, h, (0.0, 0.0, 0.0), interp=scenes.SDF_NEAREST)
    for _ in range(200):
        x = rng.uniform(1.0 / 256, 1.0 - 1.0 / 256, 3)
        i, j, k = (x / h).astype(int)
        phi, l, J = orc.sampled_sdf(tool, x)
        assert phi == float(S[i, j, k])
        g = np.array([S[i + 1, j, k] - S[i - 1, j, k], S[i, j + 1, k] - S[i, j - 1, k],
                      S[i, j, k + 1] - S[i, j, k - 1]], np.float64) / (2 * h)
        np.testing.assert_allclose(l, g / np.linalg.norm(g), atol=1e-12)
        assert not J.any()


def test_field_edges(orc):
    """Cells without complete central differences are outside the field."""
    res, h, lo = 10, 0.01, (0.0, 0.0, 0.0)
    for interp, lim in ((scenes.SDF_NEAREST, res - 1), (scenes.SDF_TRILINEAR, res - 2)):
        tool = _linear_tool(np.array([0, 1.0, 0]), 0.0, res, h, lo, interp)
        mid = 0.5 * res * h
        assert np.isfinite(orc.sampled_sdf(tool, [1.0 * h, mid, mid])[0])
        assert np.isinf(orc.sampled_sdf(tool, [0.999 * h, mid, mid])[0])
        assert np.isfinite(orc.sampled_sdf(tool, [(lim - 1e-6) * h, mid, mid])[0])
        assert np.isinf(orc.sampled_sdf(tool, [lim * h, mid, mid])[0])
        assert np.isinf(orc.sampled_sdf(tool, [mid, mid, -1.0])[0])


def _capsule_samples(res, extent, r, hl):
    h = extent / (res - 1)
    ax = -0.5 * extent + h * np.arange(res)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    q0 = X - np.clip(X, -hl, hl)
    return np.sqrt(q0 * q0 + Y * Y + Z * Z) - r, h, (-0.5 * extent,) * 3


def test_sampled_capsule_converges_to_the_analytic_one(orc):
    """A sampled capsule read back trilinearly is second-order accurate in
    the lattice spacing, in distance and in normal."""
    rng = np.random.default_rng(16)
    r, hl = 0.02, 0.05
    errs = {}
    for res in (33, 65):
        S, h, lo = _capsule_samples(res, 0.2, r, hl)
        tool = scenes.sdf_tool((0, 0, 0), S, h, lo)
        e_phi = e_n = 0.0
        rr = np.random.default_rng(17)
        for _ in range(300):
            p = rr.uniform(-0.08, 0.08, 3)
            phi_c, q, _ = orc.capsule_sdf(p, r, hl)
            if np.linalg.norm(q) < r:           # keep off the axis, where the normal turns fast
                continue
            if abs(abs(p[0]) - hl) < 0.02:      # and off the cap junctions, where the SDF is only C1
                continue
            phi, l, _ = orc.sampled_sdf(tool, p)
            e_phi = max(e_phi, abs(phi - phi_c))
            e_n = max(e_n, np.linalg.norm(l - q / np.linalg.norm(q)))
        errs[res] = (e_phi, e_n, h)
    (p1, n1, h1), (p2, n2, h2) = errs[33], errs[65]
    # bound on trilinear error: (h^2 / 8) * trace of the Hessian (<= 2 / distance to the axis)
    assert p1 <= h1 * h1 / 8 * 2 / (r - np.sqrt(3) * h1) + 1e-7
    assert p2 < p1 / 2.5 and n2 < n1 / 2.5                   # second order: ~4x per halving
    assert n2 < 0.005
    del rng


def test_trilinear_jacobian_is_the_derivative_of_the_normal(orc):
    S, h, lo = _capsule_samples(41, 0.2, 0.02, 0.05)
    tool = scenes.sdf_tool((0, 0, 0), S, h, lo)
    rng = np.random.default_rng(18)
    checked = 0
    for _ in range(60):
        s = rng.integers(2, 37, 3) + rng.uniform(0.05, 0.95, 3)   # well inside one cell
        x = np.asarray(tool.sdf_lo) + s * tool.sdf_h
        phi, l, J = orc.sampled_sdf(tool, x)
        e = 1e-6 * tool.sdf_h
        Jfd = np.stack([(orc.sampled_sdf(tool, x + e * np.eye(3)[k])[1] - orc.sampled_sdf(tool, x - e * np.eye(3)[k])[1]) / (2 * e)
                        for k in range(3)], 1)
        np.testing.assert_allclose(J, Jfd, atol=1e-5 * max(1.0, np.abs(Jfd).max()))
        checked += np.abs(J).max() > 0
    assert checked > 30


def _grid_one_node(orc, n, node, vel, tools):
    env = scenes.Env(n=n, x=np.zeros((0, 3), np.float32), v=None, C=None, F=None, E=1e4, nu=0.3, rho=1e3, V0=1e-6)
    env.tools = tools
    sim = orc.Sim(env, dt=1e-4, gravity=(0, 0, 0))
    gm = np.zeros((n, n, n)); gmv = np.zeros((n, n, n, 3))
    gm[node] = 2.0
    gmv[node] = 2.0 * np.asarray(vel, np.float64)
    gv, rec = sim.grid_update(gm, gmv, record=True)
    return gv[node], rec[(node[0] * n + node[1]) * n + node[2]]


def test_zbuffer_over_shapes(orc):
    """The collision objects table takes the nearest tool of any shape; equal
    distances go to the lowest id; sampled-SDF and box normals come out in
    world coordinates."""
    n = 32
    node = (16, 16, 16)
    xi = np.array(node) / n
    jaw = scenes.box_tool(xi + [0, 0.012, 0], (0.03, 0.0115, 0.03), u=(0, -1, 0), contact=1)   # 0.5 mm away
    S, h, lo = _capsule_samples(33, 0.2, 0.02, 0.05)
    probe = scenes.sdf_tool(xi + [0, 0.0205, 0], S, h, lo, u=(0, 1, 0), contact=1)           # ~0.5 mm inside
    out, rec = _grid_one_node(orc, n, node, np.zeros(3), [jaw, probe])
    assert rec.tool == 1
    np.testing.assert_allclose(out, [0, 1, 0], atol=1e-7)
    twin = scenes.box_tool(xi + [0, 0.012, 0], (0.03, 0.0115, 0.03), u=(0, 1, 0), contact=1)
    out, rec = _grid_one_node(orc, n, node, np.zeros(3), [jaw, twin])
    assert rec.tool == 0
    # a rotated box: slip contact normal is R times the tool-frame face normal
    th = 0.5
    R = np.array([[1, 0, 0], [0, np.cos(th), -np.sin(th)], [0, np.sin(th), np.cos(th)]])
    T = xi - R @ np.array([0.0, -0.012, 0.0])
    box = scenes.box_tool(T, (0.03, 0.0115, 0.03), u=(0, 0, 0), R=R, friction=0.0)
    out, rec = _grid_one_node(orc, n, node, np.array([0.0, 1.0, 0.0]), [box])
    assert rec.tool == 0
    np.testing.assert_allclose(np.array(rec.n), R.astype(np.float32).astype(np.float64) @ [0, -1.0, 0], atol=1e-6)


# ---------------------------------------------------------------- adjoint with the new shapes

def _W(seed, N):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((N, 3)), rng.standard_normal((N, 3)),
            rng.standard_normal((N, 3, 3)), rng.standard_normal((N, 3, 3)))


def _L(sim, W):
    st = sim.state
    return sum((a * b).sum() for a, b in zip((st.x, st.v, st.C, st.F), W))


@pytest.mark.parametrize("kind,interp", [("gripper", 1), ("sdf", 1), ("sdf", 0), ("mixed", 1)])
def test_adjoint_vs_fd_tools(orc, kind, interp):
    S, N, n = 5, 2000, 64
    sc = scenes.tool_slab_scene(51, N, kind, n=n, substeps=S, dt=1e-4, sdf_res=40, interp=interp)
    env = sc.envs[0]
    rng = np.random.default_rng(52)
    scenes.perturbed_state(rng, env, v_scale=0.05, C_scale=1.0, F_scale=0.01)
    for t in env.tools:
        t.traj = (t.traj[0] + 0.05 * rng.standard_normal((S, 3))).astype(np.float32)
    W = _W(53, N)
    sim = orc.Sim(env, dt=sc.dt)
    g = sim.adjoint(S, *W)
    assert g["flags"] == 0
    assert np.abs(g["gu"]).max() > 0

    def run(traj=None, T0=None):
        s = orc.Sim(env, dt=sc.dt)
        if traj is not None:
            s.traj[:] = traj
        if T0 is not None:
            s.T[:] = T0
        return _L(s.run(S), W)

    traj0 = sim.traj.copy()
    for t in range(len(env.tools)):
        for s_, a in [(0, 1), (S - 1, 0), (2, 2)]:
            h = 1e-6
            tp, tm = traj0.copy(), traj0.copy()
            tp[t, s_, a] += h
            tm[t, s_, a] -= h
            fd = (run(traj=tp) - run(traj=tm)) / (2 * h)
            assert g["gu"][s_, t, a] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g["gu"]).max()), (t, s_, a)
        for a in range(3):
            h = 1e-9
            T0 = sim.T.copy()
            Tp, Tm = T0.copy(), T0.copy()
            Tp[t, a] += h
            Tm[t, a] -= h
            fd = (run(T0=Tp) - run(T0=Tm)) / (2 * h)
            assert g["gT0"][t, a] == pytest.approx(fd, rel=1e-4, abs=1e-5 * np.abs(g["gT0"]).max() + 1e-7), (t, a)
    # E through the contact
    h = 1e-3
    kw = lambda d: orc.Sim(env, dt=sc.dt, E=env.E + d).run(S)
    fd = (_L(kw(h), W) - _L(kw(-h), W)) / (2 * h)
    assert g["gE"] == pytest.approx(fd, rel=2e-6, abs=1e-12)
