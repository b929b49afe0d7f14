"""Seeded synthetic scenes for the MLS-MPM tissue substep.

This module only draws inputs: particle positions, initial velocity / affine /
deformation fields, material constants and rigid-tool kinematics.  It holds none
of the method's arithmetic (no weights, no stress, no transfers), so both the
FP64 oracle and the HIP path can take their inputs from it.

Every array is drawn in float64 from ``numpy.random.default_rng(seed)`` (PCG64)
and rounded once to float32; both sides start from those float32 values.

The paper's tissue meshes and SurRoL scenes are not available, so boxes of
tissue ("particles from a distribution function", Sec. III-A) and an analytic
capsule tool stand in for them.  Geometry follows the paper's setting: a
unit-cube domain, y up, density 1000 kg/m^3 (Sec. IV-A, Fig. seq2 caption), a
64^3 grid for the 30K-particle scene (Fig. performance caption).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

CONTACT_SLIP = 0
CONTACT_STICKY = 1
TOOL_CAPSULE = 0
TOOL_BOX = 1
TOOL_SDF = 2
SDF_NEAREST = 0
SDF_TRILINEAR = 1


@dataclass
class Tool:
    """A rigid tool; pose ``R`` (world-from-tool rotation) and ``T0`` (world
    position of the tool origin at the first substep).  Shapes: capsule
    (segment of half length ``half_len`` along the tool-frame x axis, radius
    ``radius``), box (half extents ``half``, corners rounded by ``radius``),
    sampled SDF (``sdf[res][res][res]`` float32 signed distances, sample
    (i,j,k) at ``sdf_lo + (i,j,k) * sdf_h`` in the tool frame)."""
    radius: float
    half_len: float
    R: np.ndarray                 # (3, 3) float32, row-major
    T0: np.ndarray                # (3,) float32
    friction: float
    theta: float
    contact: int = CONTACT_SLIP
    traj: Optional[np.ndarray] = None   # (n_traj, 3) float32 per-substep velocity; last entry held
    shape: int = TOOL_CAPSULE
    half: tuple = (0.0, 0.0, 0.0)
    sdf: Optional[np.ndarray] = None
    sdf_h: float = 0.0
    sdf_lo: tuple = (0.0, 0.0, 0.0)
    sdf_interp: int = SDF_TRILINEAR


@dataclass
class Env:
    """One independent simulation: particles, grid, material, tools."""
    n: int                        # grid nodes per axis, dx = 1/n, domain [0,1]^3
    x: np.ndarray                 # (N, 3) float32
    v: np.ndarray                 # (N, 3) float32
    C: np.ndarray                 # (N, 3, 3) float32
    F: np.ndarray                 # (N, 3, 3) float32
    E: float
    nu: float
    rho: float
    V0: float
    tools: List[Tool] = field(default_factory=list)

    def __post_init__(self):
        # scalar inputs are FP32 values, like the arrays
        for k in ("E", "nu", "rho", "V0"):
            setattr(self, k, float(np.float32(getattr(self, k))))

    @property
    def N(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Scene:
    name: str
    envs: List[Env]
    dt: float
    substeps: int
    gravity: tuple = (0.0, -9.8, 0.0)
    bound: int = 3
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        self.dt = float(np.float32(self.dt))
        self.gravity = tuple(float(np.float32(g)) for g in self.gravity)

    @property
    def n_particles(self) -> int:
        return sum(e.N for e in self.envs)


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def _rest_state(x: np.ndarray):
    N = x.shape[0]
    v = np.zeros((N, 3), np.float32)
    C = np.zeros((N, 3, 3), np.float32)
    F = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    return v, C, F


def box_uniform(rng, n_particles: int, lo, hi) -> np.ndarray:
    """i.i.d. uniform positions in the axis-aligned box [lo, hi]."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return _f32(lo + (hi - lo) * rng.random((n_particles, 3)))


def box_stratified(rng, cells_per_axis, per_cell: int, lo, cell: float) -> np.ndarray:
    """Stratified jitter: ``per_cell`` uniform points in each cell of a
    regular lattice of cubes of edge ``cell`` starting at ``lo``."""
    cx, cy, cz = cells_per_axis
    idx = np.stack(np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij"), -1)
    idx = idx.reshape(-1, 3).astype(np.float64)
    idx = np.repeat(idx, per_cell, axis=0)
    pts = np.asarray(lo, np.float64) + (idx + rng.random(idx.shape)) * cell
    return _f32(pts)


def capsule_tool(T0, u=None, traj=None, radius=0.02, half_len=0.1, friction=0.3,
                 theta=1e-3, contact=CONTACT_SLIP, R=None) -> Tool:
    if traj is None:
        traj = np.asarray([u if u is not None else (0.0, 0.0, 0.0)], np.float64)
    return Tool(radius=float(np.float32(radius)), half_len=float(np.float32(half_len)),
                R=_f32(np.eye(3) if R is None else R), T0=_f32(T0),
                friction=float(np.float32(friction)), theta=float(np.float32(theta)),
                contact=int(contact), traj=_f32(traj))


def box_tool(T0, half, u=None, traj=None, radius=0.0, friction=0.3, theta=1e-3,
             contact=CONTACT_SLIP, R=None) -> Tool:
    """A box of half extents ``half`` (a gripper jaw's bounding box)."""
    t = capsule_tool(T0, u=u, traj=traj, radius=0.0, half_len=0.0, friction=friction, theta=theta,
                     contact=contact, R=R)
    t.radius = float(np.float32(radius))
    t.shape = TOOL_BOX
    t.half = tuple(float(h) for h in _f32(half))
    return t


def gripper_tools(center, u, close_speed=0.1, gap=0.03, jaw_half=(0.04, 0.03, 0.008), **kw):
    """Two box jaws either side of ``center`` along z, moving with ``u`` and
    closing towards each other at ``close_speed`` each."""
    c = np.asarray(center, np.float64)
    dz = np.array([0.0, 0.0, 0.5 * gap + jaw_half[2]])
    u = np.asarray(u, np.float64)
    cz = np.array([0.0, 0.0, close_speed])
    return [box_tool(c - dz, jaw_half, u=u + cz, **kw), box_tool(c + dz, jaw_half, u=u - cz, **kw)]


def probe_sdf_samples(res: int, extent: float, tip_radius=0.025, shaft_radius=0.008, shaft_len=0.1):
    """Signed-distance samples of a ball-tipped probe, the stand-in for a
    precomputed tool-mesh SDF: a ball of ``tip_radius`` at the tool origin
    and a shaft (a rod of ``shaft_radius`` from the origin up the tool-frame
    y axis, length ``shaft_len``), sampled on a ``res``^3 lattice spanning
    [-extent/2, extent/2]^3; distance of the union = min of the two.
    Returns (samples float32 [res][res][res], spacing, lattice origin)."""
    h = extent / (res - 1)
    lo = -0.5 * extent
    ax = lo + h * np.arange(res)
    Y, Z = np.meshgrid(ax, ax, indexing="ij")
    dy = Y - np.clip(Y, 0.0, shaft_len)
    out = np.empty((res, res, res), np.float32)
    for i, x in enumerate(ax):          # one x slice at a time keeps the temporaries small
        ball = np.sqrt(x * x + Y * Y + Z * Z) - tip_radius
        rod = np.sqrt(x * x + dy * dy + Z * Z) - shaft_radius
        out[i] = np.minimum(ball, rod)
    return out, float(np.float32(h)), tuple(float(v) for v in _f32((lo, lo, lo)))


def sdf_tool(T0, samples, h, lo, u=None, traj=None, interp=SDF_TRILINEAR, friction=0.3, theta=1e-3,
             contact=CONTACT_SLIP, R=None) -> Tool:
    t = capsule_tool(T0, u=u, traj=traj, radius=0.0, half_len=0.0, friction=friction, theta=theta,
                     contact=contact, R=R)
    t.shape = TOOL_SDF
    t.sdf = np.ascontiguousarray(samples, dtype=np.float32)
    t.sdf_h = float(np.float32(h))
    t.sdf_lo = tuple(float(v) for v in _f32(lo))
    t.sdf_interp = int(interp)
    return t


def rotation(rng, max_angle: float):
    """Rotation by a uniform angle in [0, max_angle] about a random axis (FP32)."""
    a = _unit(rng.standard_normal(3))
    th = rng.uniform(0.0, max_angle)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return _f32(np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def cube_scene(seed: int = 1, substeps: int = 50) -> Scene:
    """8,192 particles, stratified jitter (8^3 cells of the 32^3 grid x 16 per
    cell) in a 0.25^3 cube resting on the sticky floor band; no tool."""
    rng = np.random.default_rng(seed)
    n = 32
    dx = 1.0 / n
    lo = (0.375, 3 * dx, 0.375)
    x = box_stratified(rng, (8, 8, 8), 16, lo, dx)
    v, C, F = _rest_state(x)
    V0 = 0.25 ** 3 / x.shape[0]
    env = Env(n=n, x=x, v=v, C=C, F=F, E=5e3, nu=0.3, rho=1e3, V0=V0)
    return Scene("cube-8k-32", [env], dt=1e-4, substeps=substeps)


def slab_scene(seed: int = 2, n_particles: int = 30000, substeps: int = 1000) -> Scene:
    """Tissue slab 0.5 x 0.1 x 0.5 on the floor band of a 64^3 grid, pushed
    down by a capsule (r 0.02, segment 0.2) at 0.2 m/s, slip contact with
    friction 0.3."""
    rng = np.random.default_rng(seed)
    n = 64
    y0 = 3.0 / n
    lo, hi = (0.25, y0, 0.25), (0.75, y0 + 0.1, 0.75)
    x = box_uniform(rng, n_particles, lo, hi)
    v, C, F = _rest_state(x)
    V0 = 0.5 * 0.1 * 0.5 / n_particles
    tool = capsule_tool(T0=(0.5, y0 + 0.12, 0.5), u=(0.0, -0.2, 0.0), friction=0.3)
    env = Env(n=n, x=x, v=v, C=C, F=F, E=1e4, nu=0.35, rho=1e3, V0=V0, tools=[tool])
    return Scene(f"slab-{n_particles // 1000}k-64", [env], dt=5e-5, substeps=substeps)


def _unit(a):
    a = np.asarray(a, np.float64)
    return a / np.linalg.norm(a)


def large_slab_scene(seed: int = 3, n_particles: int = 1 << 20, substeps: int = 500) -> Scene:
    """1,048,576 particles in a 0.6 x 0.2 x 0.6 slab on a 128^3 grid; a capsule
    embedded 1 cm into the top surface pulls it with sticky contact along a
    piecewise-linear path (4 legs x 125 substeps, speed 0.2 m/s)."""
    rng = np.random.default_rng(seed)
    n = 128
    y0 = 3.0 / n
    lo, hi = (0.2, y0, 0.2), (0.8, y0 + 0.2, 0.8)
    x = box_uniform(rng, n_particles, lo, hi)
    v, C, F = _rest_state(x)
    V0 = 0.6 * 0.2 * 0.6 / n_particles
    legs, per_leg = 4, max(1, substeps // 4)
    traj = []
    for _ in range(legs):
        d = _unit((rng.uniform(-0.3, 0.3), rng.uniform(0.5, 1.0), rng.uniform(-0.3, 0.3)))
        traj.extend([0.2 * d] * per_leg)
    tool = capsule_tool(T0=(0.5, y0 + 0.2 + 0.02 - 0.01, 0.5), traj=np.asarray(traj),
                        friction=0.0, contact=CONTACT_STICKY)
    env = Env(n=n, x=x, v=v, C=C, F=F, E=2e4, nu=0.4, rho=1e3, V0=V0, tools=[tool])
    return Scene(f"large-slab-{n_particles}-128", [env], dt=2e-5, substeps=substeps)


def batched_scene(seed: int = 4, n_envs: int = 256, substeps: int = 200,
                  n_min: int = 5000, n_max: int = 50000) -> Scene:
    """``n_envs`` independent slabs: N ~ U{n_min..n_max}, grid 32^3 or 64^3,
    E ~ U[3e3, 3e4], nu ~ U[0.25, 0.45], each pushed by its own capsule at a
    constant velocity s * normalize(U[-.3,.3], -1, U[-.3,.3]), s ~ U[.05,.2]."""
    rng = np.random.default_rng(seed)
    envs = []
    for _ in range(n_envs):
        N = int(rng.integers(n_min, n_max + 1))
        n = int(rng.choice([32, 64]))
        E = float(rng.uniform(3e3, 3e4))
        nu = float(rng.uniform(0.25, 0.45))
        y0 = 3.0 / n
        x = box_uniform(rng, N, (0.25, y0, 0.25), (0.75, y0 + 0.1, 0.75))
        v, C, F = _rest_state(x)
        s = rng.uniform(0.05, 0.2)
        u = s * _unit((rng.uniform(-0.3, 0.3), -1.0, rng.uniform(-0.3, 0.3)))
        tool = capsule_tool(T0=(0.5, y0 + 0.12, 0.5), u=u, friction=0.3)
        envs.append(Env(n=n, x=x, v=v, C=C, F=F, E=E, nu=nu, rho=1e3, V0=0.5 * 0.1 * 0.5 / N, tools=[tool]))
    return Scene(f"batched-{n_envs}", envs, dt=5e-5, substeps=substeps)


def diff_scene(seed: int = 5, n_particles: int = 30000, substeps: int = 200) -> Scene:
    """The 30K slab of ``slab_scene`` with per-substep tool velocities as
    variables (initialised to (0, -0.2, 0)) and a target point for the
    centroid loss: initial centroid + (U[-.01,.01], U[-.01,0], U[-.01,.01])."""
    sc = slab_scene(seed=seed, n_particles=n_particles, substeps=substeps)
    rng = np.random.default_rng(seed + 1000)
    env = sc.envs[0]
    env.tools[0].traj = _f32(np.tile([0.0, -0.2, 0.0], (substeps, 1)))
    c0 = env.x.astype(np.float64).mean(axis=0)
    target = c0 + np.array([rng.uniform(-0.01, 0.01), rng.uniform(-0.01, 0.0),
                            rng.uniform(-0.01, 0.01)])
    sc.name = f"diff-slab-{n_particles // 1000}k-64"
    sc.extra["target"] = target
    sc.extra["checkpoint_every"] = 20
    return sc


def small_slab_scene(seed: int, n_particles: int, n: int = 32, substeps: int = 10,
                     contact: int = CONTACT_SLIP, u=(0.0, -0.2, 0.0), friction: float = 0.3,
                     dt: float = 5e-5, E: float = 1e4, nu: float = 0.35) -> Scene:
    """A reduced slab for parity and gradient tests: same shape as the 30K slab,
    fewer particles, any grid size; tool touching the top surface."""
    rng = np.random.default_rng(seed)
    y0 = 3.0 / n
    x = box_uniform(rng, n_particles, (0.25, y0, 0.25), (0.75, y0 + 0.1, 0.75))
    v, C, F = _rest_state(x)
    tool = capsule_tool(T0=(0.5, y0 + 0.12, 0.5), u=u, friction=friction, contact=contact)
    env = Env(n=n, x=x, v=v, C=C, F=F, E=E, nu=nu, rho=1e3, V0=0.5 * 0.1 * 0.5 / n_particles,
              tools=[tool])
    return Scene(f"small-slab-{n_particles}-{n}", [env], dt=dt, substeps=substeps)


def tool_slab_scene(seed: int, n_particles: int, kind: str, n: int = 32, substeps: int = 10,
                    dt: float = 5e-5, sdf_res: int = 48, interp: int = SDF_TRILINEAR,
                    contact: int = CONTACT_SLIP, friction: float = 0.3) -> Scene:
    """The reduced slab of ``small_slab_scene`` pressed by other tools:
    ``kind`` "gripper" (two closing box jaws, slightly rotated), "sdf" (a
    sampled ball-tipped probe, tilted, lattice ``sdf_res``^3 over 0.24 m) or
    "mixed" (the probe and one jaw overlapping, for the z-buffer)."""
    sc = small_slab_scene(seed, n_particles, n=n, substeps=substeps, dt=dt)
    rng = np.random.default_rng(seed + 77)
    env = sc.envs[0]
    y0 = 3.0 / n
    top = y0 + 0.1
    # tool origins off the lattice of nodes
    jitter = rng.uniform(-0.3, 0.3, 3) / n
    kw = dict(friction=friction, contact=contact)
    tools = []
    if kind in ("gripper", "mixed"):
        R = rotation(rng, 0.3)
        jaws = gripper_tools((0.5 + jitter[0], top + 0.01, 0.5 + jitter[2]), (0.0, -0.2, 0.0), R=R, **kw)
        tools += jaws if kind == "gripper" else jaws[:1]
    if kind in ("sdf", "mixed"):
        S, h, lo = probe_sdf_samples(sdf_res, 0.24)
        tools.append(sdf_tool((0.5 - jitter[0], top + 0.005, 0.5 - jitter[2]), S, h, lo, u=(0.02, -0.25, 0.0),
                              interp=interp, R=rotation(rng, 0.4), **kw))
    env.tools = tools
    sc.name = f"{kind}-slab-{n_particles}-{n}"
    return sc


def slab_tool_scene(kind: str, seed: int = 2, n_particles: int = 30000, substeps: int = 1000,
                    sdf_res: int = 256, interp: int = SDF_TRILINEAR) -> Scene:
    """The 30K slab with its capsule replaced by a box gripper ("gripper":
    two jaws 1 cm into the top surface, pushing at 0.2 m/s and closing at
    0.1 m/s each) or a sampled ball-tipped probe ("sdf": ``sdf_res``^3
    samples at spacing 1/256 m around the tool origin, so 256 samples span
    the unit domain, tip 2 cm into the top surface, pushing at 0.2 m/s)."""
    sc = slab_scene(seed=seed, n_particles=n_particles, substeps=substeps)
    top = 3.0 / 64 + 0.1
    if kind == "gripper":
        tools = gripper_tools((0.5, top + 0.02, 0.5), (0.0, -0.2, 0.0))
    elif kind == "sdf":
        S, h, lo = probe_sdf_samples(sdf_res, (sdf_res - 1) / 256.0)
        tools = [sdf_tool((0.5, top + 0.005, 0.5), S, h, lo, u=(0.0, -0.2, 0.0), interp=interp)]
    else:
        raise ValueError(kind)
    sc.envs[0].tools = tools
    sc.name = f"slab-{kind}-{n_particles // 1000}k-64"
    return sc


def perturbed_state(rng, env: Env, v_scale=0.1, C_scale=2.0, F_scale=0.02):
    """Random non-rest state (velocity, affine field, deformation near I) for
    tests that need every term of the substep to be active."""
    N = env.N
    env.v = _f32(v_scale * rng.standard_normal((N, 3)))
    env.C = _f32(C_scale * rng.standard_normal((N, 3, 3)))
    env.F = _f32(np.eye(3) + F_scale * rng.standard_normal((N, 3, 3)))
    return env


SCENES = {
    "cube": cube_scene,
    "slab": slab_scene,
    "large": large_slab_scene,
    "batched": batched_scene,
    "diff": diff_scene,
}
