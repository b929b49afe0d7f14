"""ctypes shim over the FP64 C oracle (``mpm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  Never imported by the product package.

Arrays cross as contiguous float64 numpy arrays in the oracle's own layout:
particles AoS (x (N,3), v (N,3), C (N,3,3), F (N,3,3)), grids dense
(n,n,n[,3]) with node (i,j,k) at position (i,j,k)/n.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpm_oracle.c")
LIB = os.path.join(HERE, "libmpm_oracle.so")

FLAG_OUT_OF_DOMAIN = 1
FLAG_INVERTED = 2
FLAG_NONFINITE = 4
J_MIN = 1e-6


CFLAGS = ["-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True, out: str = LIB, native: bool = False, extra=()) -> str:
    """Compile the oracle with gcc: -O3 and OpenMP (for orc_run_threads), ISO C
    (so no floating-point contraction and no fast-math).  native=True adds
    -march=native, for a library built and timed on the same host."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        flags = CFLAGS + (["-march=native"] if native else []) + list(extra)
        subprocess.check_call(["gcc", *flags, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, out)
    return out


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (e.g. a
    -march=native build made on the timing host); call before any other use."""
    global _lib, LIB
    _lib = None
    LIB = path


class Params(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("bound", ct.c_int32), ("n_tools", ct.c_int32), ("pad", ct.c_int32),
                ("dt", ct.c_double), ("g", ct.c_double * 3),
                ("E", ct.c_double), ("nu", ct.c_double), ("rho", ct.c_double), ("V0", ct.c_double)]


class ToolC(ct.Structure):
    _fields_ = [("contact", ct.c_int32), ("shape", ct.c_int32),
                ("radius", ct.c_double), ("half_len", ct.c_double), ("friction", ct.c_double),
                ("theta", ct.c_double), ("R", ct.c_double * 9), ("half", ct.c_double * 3),
                ("sdf_h", ct.c_double), ("sdf_lo", ct.c_double * 3), ("sdf_res", ct.c_int32),
                ("sdf_interp", ct.c_int32), ("sdf", ct.c_void_p)]


class NodeRec(ct.Structure):
    _fields_ = [("vhat", ct.c_double * 3), ("n", ct.c_double * 3), ("q", ct.c_double * 3),
                ("tool", ct.c_int32), ("branch", ct.c_int32), ("wall", ct.c_int32), ("interior", ct.c_int32),
                ("xr", ct.c_double * 3)]


_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ct.CDLL(LIB)
        P, T = ct.POINTER(Params), ct.POINTER(ToolC)
        L.orc_lame.argtypes = [ct.c_double, ct.c_double, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        L.orc_weights.argtypes = [_D, ct.c_double, ct.POINTER(ct.c_int), _D, _D, _D]
        L.orc_kirchhoff.argtypes = [_D, ct.c_double, ct.c_double, _D]
        L.orc_kirchhoff.restype = ct.c_uint32
        L.orc_capsule_sdf.argtypes = [_D, ct.c_double, ct.c_double, _D, ct.POINTER(ct.c_int)]
        L.orc_capsule_sdf.restype = ct.c_double
        L.orc_box_sdf.argtypes = [_D, _D, ct.c_double, _D, _D]
        L.orc_box_sdf.restype = ct.c_double
        L.orc_sampled_sdf.argtypes = [T, _D, _D, _D]
        L.orc_sampled_sdf.restype = ct.c_double
        L.orc_p2g.argtypes = [P, ct.c_int32, _D, _D, _D, _D, _D, _D]
        L.orc_p2g.restype = ct.c_uint32
        L.orc_grid_update.argtypes = [P, T, ct.c_void_p, ct.c_void_p, _D, _D, _D, ct.c_void_p]
        L.orc_g2p.argtypes = [P, ct.c_int32, _D, _D, _D, _D, _D]
        L.orc_g2p.restype = ct.c_uint32
        L.orc_run.argtypes = [P, T, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p,
                              ct.c_int32, _D, _D, _D, _D]
        L.orc_run.restype = ct.c_uint32
        L.orc_run_threads.argtypes = [P, T, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p,
                                      ct.c_int32, _D, _D, _D, _D, ct.c_int32]
        L.orc_run_threads.restype = ct.c_uint32
        L.orc_adjoint.argtypes = [P, T, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_int32,
                                  _D, _D, _D, _D, _D, _D, _D, _D,
                                  ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.c_void_p, ct.c_void_p]
        L.orc_adjoint.restype = ct.c_uint32
        L.orc_g2p_adjoint.argtypes = [P, ct.c_int32, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_grid_adjoint.argtypes = [P, T, _D, _D, _D, ct.c_void_p, _D, _D, _D, ct.c_void_p, ct.c_void_p]
        L.orc_p2g_adjoint.argtypes = [P, ct.c_int32, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                      ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        L.orc_mc_case.argtypes = [ct.c_int, ct.c_void_p]
        L.orc_mc_case.restype = ct.c_int
        L.orc_surface.argtypes = [ct.c_int32, ct.c_double, _D, ct.c_double, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                  ct.c_int64]
        L.orc_surface.restype = ct.c_int64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


@dataclass
class State:
    """FP64 particle state (AoS) of one environment."""
    x: np.ndarray
    v: np.ndarray
    C: np.ndarray
    F: np.ndarray

    def copy(self):
        return State(self.x.copy(), self.v.copy(), self.C.copy(), self.F.copy())

    @staticmethod
    def from_env(env):
        f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64))
        return State(f(env.x), f(env.v), f(env.C), f(env.F))


class Sim:
    """One environment of a scene, simulated by the oracle."""

    def __init__(self, env, dt, gravity=(0.0, -9.8, 0.0), bound=3, E=None, nu=None):
        self.env = env
        self.n = env.n
        self.P = Params(n=env.n, bound=bound, n_tools=len(env.tools), pad=0, dt=float(dt),
                        g=(ct.c_double * 3)(*map(float, gravity)),
                        E=float(env.E if E is None else E), nu=float(env.nu if nu is None else nu),
                        rho=float(env.rho), V0=float(env.V0))
        nt = max(1, len(env.tools))
        self.tools = (ToolC * nt)()
        self._sdf = []      # keeps the sample arrays the tool records point to alive
        for i, t in enumerate(env.tools):
            self.tools[i] = tool_record(t, self._sdf)
        self.n_traj = max([t.traj.shape[0] for t in env.tools], default=1)
        self.traj = np.zeros((nt, self.n_traj, 3))
        for i, t in enumerate(env.tools):
            tr = np.asarray(t.traj, np.float64)
            self.traj[i, :tr.shape[0]] = tr
            self.traj[i, tr.shape[0]:] = tr[-1]
        self.T = np.zeros((nt, 3))
        for i, t in enumerate(env.tools):
            self.T[i] = np.asarray(t.T0, np.float64)
        self.s = 0
        self.state = State.from_env(env)
        self.flags = 0

    @property
    def n_tools(self):
        return len(self.env.tools)

    def u_at(self, s):
        k = min(s, self.n_traj - 1)
        return np.ascontiguousarray(self.traj[:, k, :])

    def run(self, S, threads=None):
        """S substeps.  threads > 1: orc_run_threads on that many threads (the
        same result bit for bit, in less wall time)."""
        st = self.state
        if threads and threads > 1:
            f = lib().orc_run_threads(ct.byref(self.P), self.tools, _ptr(self.traj), self.n_traj, self.s, S,
                                      _ptr(self.T), st.x.shape[0], st.x, st.v, st.C, st.F, int(threads))
        else:
            f = lib().orc_run(ct.byref(self.P), self.tools, _ptr(self.traj), self.n_traj, self.s, S,
                              _ptr(self.T), st.x.shape[0], st.x, st.v, st.C, st.F)
        self.flags |= f
        self.s += S
        return self

    # --- stage-level access -------------------------------------------------
    def p2g(self):
        st, n = self.state, self.n
        gm = np.zeros((n, n, n))
        gmv = np.zeros((n, n, n, 3))
        f = lib().orc_p2g(ct.byref(self.P), st.x.shape[0], st.x, st.v, st.C, st.F, gm, gmv)
        self.flags |= f
        return gm, gmv

    def grid_update(self, gm, gmv, record=False):
        n = self.n
        gv = np.zeros((n, n, n, 3))
        T = np.ascontiguousarray(self.T)
        u = self.u_at(self.s)
        rec = (NodeRec * (n * n * n))() if record else None
        lib().orc_grid_update(ct.byref(self.P), self.tools, _ptr(T), _ptr(u),
                              np.ascontiguousarray(gm), np.ascontiguousarray(gmv), gv,
                              ct.cast(rec, ct.c_void_p) if record else None)
        return (gv, rec) if record else gv

    def g2p(self, gv):
        st = self.state
        self.flags |= lib().orc_g2p(ct.byref(self.P), st.x.shape[0], st.x, st.v, st.C, st.F,
                                    np.ascontiguousarray(gv))
        u = self.u_at(self.s)
        self.T[:self.n_tools] += self.P.dt * u[:self.n_tools]
        self.s += 1

    # --- stage-level adjoints (the reverse of one stage, from the forward's inputs)
    def g2p_adjoint(self, gv, xbar, vbar, Cbar, Fbar):
        """Reverse of G2P + advection + F update from the current state (the
        stage's input) and node velocities gv; seeds are the adjoints of the
        stage's output.  Returns (xbar, vbar, Cbar, Fbar) of the input and the
        node-velocity adjoint gvbar (n, n, n, 3)."""
        st, n = self.state, self.n
        c = lambda a, shp: np.ascontiguousarray(np.asarray(a, np.float64).reshape(shp)).copy()
        N = st.x.shape[0]
        xb, vb, Cb, Fb = c(xbar, (N, 3)), c(vbar, (N, 3)), c(Cbar, (N, 3, 3)), c(Fbar, (N, 3, 3))
        gvb = np.zeros((n, n, n, 3))
        lib().orc_g2p_adjoint(ct.byref(self.P), N, st.x, st.F, np.ascontiguousarray(gv, np.float64),
                              xb, vb, Cb, Fb, gvb)
        return xb, vb, Cb, Fb, gvb

    def grid_adjoint(self, gm, gmv, rec, gvbar, u=None):
        """Reverse of the grid operation with the node records `rec` of the
        forward (grid_update(..., record=True)); returns (gmbar, gmvbar,
        ubar [n_tools][3], Tbar [n_tools][3])."""
        n, nt = self.n, max(1, self.n_tools)
        u = self.u_at(self.s) if u is None else np.ascontiguousarray(np.asarray(u, np.float64).reshape(-1, 3))
        gmb, gmvb = np.zeros((n, n, n)), np.zeros((n, n, n, 3))
        ub, Tb = np.zeros((nt, 3)), np.zeros((nt, 3))
        lib().orc_grid_adjoint(ct.byref(self.P), self.tools, np.ascontiguousarray(u), np.ascontiguousarray(gm),
                               np.ascontiguousarray(gmv), ct.cast(rec, ct.c_void_p),
                               np.ascontiguousarray(gvbar, np.float64), gmb, gmvb, _ptr(ub), _ptr(Tb))
        return gmb, gmvb, ub[:self.n_tools], Tb[:self.n_tools]

    def p2g_adjoint(self, gmbar, gmvbar):
        """Reverse of P2G and the stress from the current state; returns the
        state adjoints (xbar, vbar, Cbar, Fbar) and (mubar, lambar)."""
        st = self.state
        N = st.x.shape[0]
        xb, vb, Cb, Fb = np.zeros((N, 3)), np.zeros((N, 3)), np.zeros((N, 3, 3)), np.zeros((N, 3, 3))
        mub, lamb = ct.c_double(0.0), ct.c_double(0.0)
        lib().orc_p2g_adjoint(ct.byref(self.P), N, st.x, st.v, st.C, st.F, np.ascontiguousarray(gmbar, np.float64),
                              np.ascontiguousarray(gmvbar, np.float64), xb, vb, Cb, Fb, ct.byref(mub),
                              ct.byref(lamb))
        return xb, vb, Cb, Fb, mub.value, lamb.value

    def adjoint(self, S, xbar=None, vbar=None, Cbar=None, Fbar=None):
        """Reverse-mode gradients of S substeps from the current state.  Seeds
        are adjoints of the final state; returns a dict with the adjoints of
        the initial state, dL/dE, dL/dnu, dL/du_s ([S][n_tools][3]) and dL/dT0."""
        st = self.state
        N = st.x.shape[0]
        z = lambda shp, a: np.ascontiguousarray(np.zeros(shp) if a is None else np.asarray(a, np.float64).copy())
        xb, vb, Cb, Fb = z((N, 3), xbar), z((N, 3), vbar), z((N, 3, 3), Cbar), z((N, 3, 3), Fbar)
        gE, gnu = ct.c_double(0.0), ct.c_double(0.0)
        nt = max(1, self.n_tools)
        gu = np.zeros((S, nt, 3))
        gT0 = np.zeros((nt, 3))
        T0 = np.ascontiguousarray(self.T)
        f = lib().orc_adjoint(ct.byref(self.P), self.tools, _ptr(self.traj), self.n_traj, S, _ptr(T0), N,
                              st.x, st.v, st.C, st.F, xb, vb, Cb, Fb, ct.byref(gE), ct.byref(gnu),
                              _ptr(gu), _ptr(gT0))
        return dict(xbar=xb, vbar=vb, Cbar=Cb, Fbar=Fb, gE=gE.value, gnu=gnu.value,
                    gu=gu[:, :self.n_tools], gT0=gT0[:self.n_tools], flags=f)


# --- small helpers used by tests --------------------------------------------

def tool_record(t, keep):
    """The oracle's record of a scenes.Tool; sample arrays are appended to keep."""
    rec = ToolC(contact=int(t.contact), shape=int(t.shape), radius=float(t.radius), half_len=float(t.half_len),
                friction=float(t.friction), theta=float(t.theta),
                R=(ct.c_double * 9)(*np.asarray(t.R, np.float64).reshape(-1)),
                half=(ct.c_double * 3)(*np.asarray(t.half, np.float64)))
    if t.sdf is not None:
        a = np.ascontiguousarray(t.sdf, dtype=np.float32)
        keep.append(a)
        rec.sdf = a.ctypes.data
        rec.sdf_res = a.shape[0]
        rec.sdf_h = float(t.sdf_h)
        rec.sdf_lo = (ct.c_double * 3)(*np.asarray(t.sdf_lo, np.float64))
        rec.sdf_interp = int(t.sdf_interp)
    return rec


def box_sdf(xref, half, radius=0.0):
    """(phi, l, Jl) of a box tool at tool-frame point xref."""
    l, J = np.zeros(3), np.zeros(9)
    phi = lib().orc_box_sdf(np.ascontiguousarray(np.asarray(xref, np.float64)),
                            np.ascontiguousarray(np.asarray(half, np.float64)), float(radius), l, J)
    return phi, l, J.reshape(3, 3)


def sampled_sdf(tool, xref):
    """(phi, l, Jl) of a sampled-SDF tool (scenes.Tool) at tool-frame point xref."""
    keep = []
    rec = tool_record(tool, keep)
    l, J = np.zeros(3), np.zeros(9)
    phi = lib().orc_sampled_sdf(ct.byref(rec), np.ascontiguousarray(np.asarray(xref, np.float64)), l, J)
    return phi, l, J.reshape(3, 3)

def lame(E, nu):
    mu, lam = ct.c_double(), ct.c_double()
    lib().orc_lame(E, nu, ct.byref(mu), ct.byref(lam))
    return mu.value, lam.value


def weights(x, inv_dx, with_grad=False):
    x = np.ascontiguousarray(np.asarray(x, np.float64))
    base = (ct.c_int * 3)()
    fx = np.zeros(3)
    w = np.zeros((3, 3))
    dw = np.zeros((3, 3))
    lib().orc_weights(x, float(inv_dx), base, fx, w, dw)
    out = (np.array(list(base)), fx, w)
    return out + (dw,) if with_grad else out


def kirchhoff(F, mu, lam):
    tau = np.zeros(9)
    f = lib().orc_kirchhoff(np.ascontiguousarray(np.asarray(F, np.float64).reshape(9)), mu, lam, tau)
    return tau.reshape(3, 3), f


def capsule_sdf(xref, radius, half_len):
    q = np.zeros(3)
    inside = ct.c_int()
    phi = lib().orc_capsule_sdf(np.ascontiguousarray(np.asarray(xref, np.float64)), radius, half_len, q,
                                ct.byref(inside))
    return phi, q, bool(inside.value)


def mc_case(mask):
    """Triangles of one marching-cubes cell case as edge triples, (T, 3)."""
    tri = np.zeros((12, 3), np.int32)
    nt = lib().orc_mc_case(int(mask), tri.ctypes.data_as(ct.c_void_p))
    if nt < 0:
        raise RuntimeError(f"case {mask}: face segments do not close")
    return tri[:nt]


def surface(rho, h, iso):
    """Iso-surface rho = iso of a node field rho (n, n, n): triangles (T, 3, 3)
    in cell order, triangles per cell ((n-1)^3,), edge ids (T, 3)."""
    rho = np.ascontiguousarray(np.asarray(rho, np.float64))
    n = rho.shape[0]
    cells = np.zeros((n - 1) ** 3, np.int32)
    total = lib().orc_surface(n, float(h), rho, float(iso), cells.ctypes.data_as(ct.c_void_p), None, None, 0)
    if total < 0:
        raise RuntimeError("face segments do not close")
    tris = np.zeros((max(total, 1), 3, 3))
    edges = np.zeros((max(total, 1), 3), np.int32)
    lib().orc_surface(n, float(h), rho, float(iso), None, edges.ctypes.data_as(ct.c_void_p),
                      tris.ctypes.data_as(ct.c_void_p), total)
    return tris[:total], cells, edges[:total]
