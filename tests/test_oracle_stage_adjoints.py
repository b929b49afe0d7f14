"""Per-stage transpose (dot-product) tests of the oracle's adjoint.

For each stage f of the substep (G2P + advection + F update, the grid
operation, P2G with the stress) and random directions d, l:
    < J d, l >  =  < d, J^T l >
where J^T l comes from the stage's hand-written reverse (orc_g2p_adjoint,
orc_grid_adjoint, orc_p2g_adjoint, the functions orc_adjoint chains) and
J d from FP64 central differences of the stage's forward function
(orc_g2p, orc_grid_update, orc_p2g).  The identity is exact; central
differences with a relative step of 1e-6 are good to about 1e-9 here, so the
two sides are held to 1e-7 relative.  A dropped term, a wrong sign or a
transposed operand in any reverse stage breaks one of these."""
import ctypes as ct

import numpy as np
import pytest

from paper_2402_01181_amd import scenes

TOL = 1e-7


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _scene(contact=scenes.CONTACT_SLIP):
    sc = scenes.small_slab_scene(seed=41, n_particles=600, n=32, substeps=4, contact=contact, u=(0.1, -0.6, 0.05),
                                 dt=1e-4, friction=0.05)
    env = sc.envs[0]
    env.tools[0].T0 = (env.tools[0].T0 - np.array([0, 0.045, 0])).astype(np.float32)
    scenes.perturbed_state(np.random.default_rng(4), env, v_scale=0.3, C_scale=2.0, F_scale=0.02)
    return sc


def _oracle(orc, sc):
    return orc.Sim(sc.envs[0], dt=sc.dt, gravity=sc.gravity, bound=sc.bound)


def _g2p_out(o, state, gv):
    o.state = state.copy()
    s0, T0 = o.s, o.T.copy()
    o.g2p(gv)
    o.s, o.T = s0, T0
    st = o.state
    return st.x.copy(), st.v.copy(), st.C.copy(), st.F.copy()


def test_g2p_stage_transpose(orc):
    sc = _scene()
    o = _oracle(orc, sc)
    rng = np.random.default_rng(1)
    base = o.state.copy()
    gm, gmv = o.p2g()
    gv = o.grid_update(gm, gmv)
    n = o.n
    dx, dF, dgv = rng.standard_normal(base.x.shape) / n, rng.standard_normal(base.F.shape), rng.standard_normal(gv.shape)
    lam = [rng.standard_normal(a.shape) for a in (base.x, base.v, base.C, base.F)]
    h = 1e-6

    def at(t):
        st = base.copy()
        st.x = st.x + t * dx
        st.F = st.F + t * dF
        return _g2p_out(o, st, gv + t * dgv)

    plus, minus = at(h), at(-h)
    jd_l = sum(((p - m) / (2 * h) * l).sum() for p, m, l in zip(plus, minus, lam))
    o.state = base.copy()
    xb, vb, Cb, Fb, gvb = o.g2p_adjoint(gv, *lam)
    d_jtl = (dx * xb).sum() + (dF * Fb).sum() + (dgv * gvb).sum()
    assert np.abs(vb).max() == 0 and np.abs(Cb).max() == 0     # v and C are overwritten by the stage
    assert _rel(jd_l, d_jtl) <= TOL, (jd_l, d_jtl)


@pytest.mark.parametrize("contact", [scenes.CONTACT_SLIP, scenes.CONTACT_STICKY])
def test_grid_stage_transpose(orc, contact):
    sc = _scene(contact)
    o = _oracle(orc, sc)
    rng = np.random.default_rng(2)
    gm, gmv = o.p2g()
    gv, rec = o.grid_update(gm, gmv, record=True)
    tools = np.array([r.tool for r in rec])
    branches = np.array([r.branch for r in rec])
    assert (tools >= 0).sum() > 10, "the tool must touch nodes"
    if contact == scenes.CONTACT_SLIP:
        assert (branches == 1).sum() > 5, "some nodes must take the friction branch"
    mask = gm > 0
    dgm = rng.standard_normal(gm.shape) * gm * mask * 0.1
    dgmv = rng.standard_normal(gmv.shape) * gm.max() * 0.01
    du = rng.standard_normal((1, 3))
    dT = rng.standard_normal((1, 3)) * 1e-2
    lam = rng.standard_normal(gv.shape)
    h = 1e-6
    u0 = o.u_at(o.s).copy()
    T0 = o.T.copy()
    k = min(o.s, o.n_traj - 1)

    def at(t):
        o.traj[0, k] = u0[0] + t * du[0]
        o.T = T0 + t * dT
        g, r = o.grid_update(gm + t * dgm, gmv + t * dgmv, record=True)
        assert np.array_equal(np.array([q.branch for q in r]), branches), "step changed a contact branch"
        return g

    jd_l = ((at(h) - at(-h)) / (2 * h) * lam).sum()
    o.traj[0, k] = u0[0]
    o.T = T0
    gmb, gmvb, ub, Tb = o.grid_adjoint(gm, gmv, rec, lam, u=u0)
    d_jtl = (dgm * gmb).sum() + (dgmv * gmvb).sum() + (du * ub).sum() + (dT * Tb).sum()
    assert _rel(jd_l, d_jtl) <= TOL, (jd_l, d_jtl)
    assert np.abs(Tb).max() > 0 if contact == scenes.CONTACT_SLIP else True


def test_p2g_stage_transpose(orc):
    sc = _scene()
    o = _oracle(orc, sc)
    rng = np.random.default_rng(3)
    base = o.state.copy()
    n = o.n
    d = [rng.standard_normal(base.x.shape) / n, rng.standard_normal(base.v.shape),
         rng.standard_normal(base.C.shape), rng.standard_normal(base.F.shape) * 0.1]
    gm0, _ = o.p2g()
    lam_m = rng.standard_normal(gm0.shape)
    lam_mv = rng.standard_normal(gm0.shape + (3,))
    h = 1e-6

    def at(t, E=None, nu=None):
        st = base.copy()
        st.x, st.v, st.C, st.F = st.x + t * d[0], st.v + t * d[1], st.C + t * d[2], st.F + t * d[3]
        q = orc.Sim(sc.envs[0], dt=sc.dt, gravity=sc.gravity, bound=sc.bound, E=E, nu=nu)
        q.state = st
        return q.p2g()

    (mp, mvp), (mm, mvm) = at(h), at(-h)
    jd_l = ((mp - mm) / (2 * h) * lam_m).sum() + ((mvp - mvm) / (2 * h) * lam_mv).sum()
    o.state = base.copy()
    xb, vb, Cb, Fb, mub, lamb = o.p2g_adjoint(lam_m, lam_mv)
    d_jtl = sum((di * bi).sum() for di, bi in zip(d, (xb, vb, Cb, Fb)))
    assert _rel(jd_l, d_jtl) <= TOL, (jd_l, d_jtl)

    # the Lame-parameter adjoints, through E and nu (the Lame relation by central differences too)
    E, nu = float(sc.envs[0].E), float(sc.envs[0].nu)
    for dE, dnu in ((E * 1e-6, 0.0), (0.0, 1e-7)):
        (mp, mvp), (mm, mvm) = at(0.0, E + dE, nu + dnu), at(0.0, E - dE, nu - dnu)
        jd_l = ((mp - mm) / 2 * lam_m).sum() + ((mvp - mvm) / 2 * lam_mv).sum()
        (mu1, la1), (mu0, la0) = orc.lame(E + dE, nu + dnu), orc.lame(E - dE, nu - dnu)
        d_jtl = (mu1 - mu0) / 2 * mub + (la1 - la0) / 2 * lamb
        assert _rel(jd_l, d_jtl) <= 1e-6, (dE, dnu, jd_l, d_jtl)
