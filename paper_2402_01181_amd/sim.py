"""Python face of the library: a ``Sim`` that owns one C context.

torch provides the device memory (workspace, initial state, material table,
tool trajectories, gradient buffers) and the stream; the C ABI does the rest.
"""
from __future__ import annotations

import ctypes as ct
from typing import Dict, Optional

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _soa(arrays, comps):
    """Concatenate per-env AoS float32 arrays into one [comps][Ntot] array."""
    return np.ascontiguousarray(np.concatenate([np.asarray(a, np.float32).reshape(-1, comps) for a in arrays], 0).T)


class Sim:
    """All environments of a scene in one context on one GPU."""

    def __init__(self, scene, device="cuda", max_tape: int = 0, checkpoint_every: int = 20,
                 options: Optional[Dict[int, int]] = None, stream=None, static_workspace: bool = False,
                 hold_tape: bool = False):
        """static_workspace: create the context with mpm_create_static (the
        library's own per-device workspace of STATIC_WORKSPACE_BYTES; one such
        context per device at a time) instead of a torch-allocated workspace.
        hold_tape: keep every segment's recomputed tape of a recording, so the
        adjoint that follows it does not recompute (mpm_desc.hold_tape)."""
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (there is no CPU path)")
        self.lib = L.load()
        self.scene = scene
        self.device = torch.device(device)
        envs = scene.envs
        self.n_envs = len(envs)
        self.max_tools = max([len(e.tools) for e in envs], default=0)
        self.np = np.array([e.N for e in envs], np.int32)
        self.gn = np.array([e.n for e in envs], np.int32)
        self.pofs = np.concatenate([[0], np.cumsum(self.np)]).astype(np.int64)
        dev = self.device
        t = lambda a: torch.from_numpy(a).to(dev)
        self._x0 = t(_soa([e.x for e in envs], 3))
        self._v0 = t(_soa([e.v for e in envs], 3))
        self._C0 = t(_soa([e.C for e in envs], 9))
        self._F0 = t(_soa([e.F for e in envs], 9))
        self.material = t(np.array([[e.E, e.nu, e.rho, e.V0] for e in envs], np.float32))
        self._np_c = (ct.c_int32 * self.n_envs)(*self.np.tolist())
        self._gn_c = (ct.c_int32 * self.n_envs)(*self.gn.tolist())
        self.desc = L.MpmDesc(
            n_envs=self.n_envs, n_particles=self._np_c, grid_n=self._gn_c, dt=float(scene.dt),
            gravity=(ct.c_float * 3)(*scene.gravity), bound=int(scene.bound), max_tools=self.max_tools,
            checkpoint_every=int(checkpoint_every), max_tape_substeps=int(max_tape),
            x0=self._x0.data_ptr(), v0=self._v0.data_ptr(), C0=self._C0.data_ptr(), F0=self._F0.data_ptr(),
            material=self.material.data_ptr(), hold_tape=int(bool(hold_tape)))
        size = self.lib.mpm_workspace_size(ct.byref(self.desc))
        if size == 0:
            raise L.MpmError(L.MPM_E_ARG, self.lib.mpm_last_error(None).decode())
        self.workspace_bytes = size
        self.static_workspace = bool(static_workspace)
        self.workspace = None if self.static_workspace else torch.empty(size + 256, dtype=torch.uint8, device=dev)
        self.max_tape = int(max_tape)
        self.options = dict(options or {})
        self.traj = {}
        self._sdf = {}        # id(samples) -> (host array, device copy) of sampled-SDF tools
        self.ctx = ct.c_void_p()
        self._create(stream)

    def _create(self, stream=None):
        if self.static_workspace:
            with torch.cuda.device(self.device):
                L.check(self.lib.mpm_create_static(ct.byref(self.desc), _stream_ptr(stream), ct.byref(self.ctx)))
        else:
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            L.check(self.lib.mpm_create(ct.byref(self.desc), ct.c_void_p(aligned), self.workspace_bytes,
                                        _stream_ptr(stream), ct.byref(self.ctx)))
        for e, env in enumerate(self.scene.envs):
            for k, tool in enumerate(env.tools):
                self.set_tool(e, k, tool, traj=self.traj.get((e, k)))
        for opt, val in self.options.items():
            self.set_option(opt, val)

    def reset(self, stream=None):
        """Back to the initial state (same workspace, tools at T0, current
        material table and trajectories)."""
        self.close()
        self._create(stream)

    # ------------------------------------------------------------------ control
    def set_tool(self, env, slot, tool, traj=None):
        if isinstance(traj, torch.Tensor):
            u = traj.detach().to(self.device, torch.float32).contiguous()
        else:
            u = torch.from_numpy(np.ascontiguousarray(np.asarray(tool.traj if traj is None else traj,
                                                                 np.float32))).to(self.device)
        self.traj[(env, slot)] = u
        shape = int(getattr(tool, "shape", L.TOOL_CAPSULE))
        td = L.MpmTool(shape=shape, contact=int(tool.contact), radius=tool.radius,
                       half_len=tool.half_len, friction=tool.friction, theta=tool.theta,
                       R=(ct.c_float * 9)(*np.asarray(tool.R, np.float32).reshape(-1).tolist()),
                       T0=(ct.c_float * 3)(*np.asarray(tool.T0, np.float32).tolist()),
                       half=(ct.c_float * 3)(*np.asarray(getattr(tool, "half", (0, 0, 0)), np.float32).tolist()))
        if shape == L.TOOL_SDF:
            # device copy of the samples, shared by every slot given the same array
            key = id(tool.sdf)
            if key not in self._sdf:
                self._sdf[key] = (tool.sdf, torch.from_numpy(np.ascontiguousarray(tool.sdf, np.float32)).to(self.device))
            S = self._sdf[key][1]
            td.sdf = S.data_ptr()
            td.sdf_res = int(S.shape[0])
            td.sdf_interp = int(tool.sdf_interp)
            td.sdf_h = float(tool.sdf_h)
            td.sdf_lo = (ct.c_float * 3)(*np.asarray(tool.sdf_lo, np.float32).tolist())
        L.check(self.lib.mpm_set_tool(self.ctx, env, slot, ct.byref(td), ct.c_void_p(u.data_ptr()), u.shape[0]),
                self.ctx)

    def set_option(self, option, value):
        L.check(self.lib.mpm_set_option(self.ctx, int(option), int(value)), self.ctx)
        self.options[int(option)] = int(value)

    def step(self, n=1, record_tape=False, stream=None):
        L.check(self.lib.mpm_substep(self.ctx, int(n), 1 if record_tape else 0, _stream_ptr(stream)), self.ctx)

    def stage(self, stage, stream=None):
        L.check(self.lib.mpm_run_stage(self.ctx, int(stage), _stream_ptr(stream)), self.ctx)

    def adjoint(self, n, xbar=None, vbar=None, Cbar=None, Fbar=None, stream=None):
        """Reverse the last n recorded substeps.  Seeds are adjoints of the
        current state as [comps][Ntot] tensors in the original particle order
        (environments concatenated); None means zero.  Returns a dict of
        device tensors: xbar0, vbar0, Cbar0, Fbar0 ([comps][Ntot]), gE, gnu
        ([n_envs], float64), gu ([n_envs][max_tools][n][3]), gT
        ([n_envs][max_tools][3])."""
        N, dev = int(self.pofs[-1]), self.device
        def seed(a, comps):
            if a is None:
                return None
            t = torch.as_tensor(a, dtype=torch.float32, device=dev).reshape(comps, N).contiguous()
            return t
        seeds = [seed(xbar, 3), seed(vbar, 3), seed(Cbar, 9), seed(Fbar, 9)]
        outs = [torch.empty((c, N), dtype=torch.float32, device=dev) for c in (3, 3, 9, 9)]
        nt = max(1, self.max_tools)
        gE = torch.empty(self.n_envs, dtype=torch.float64, device=dev)
        gnu = torch.empty(self.n_envs, dtype=torch.float64, device=dev)
        gu = torch.zeros((self.n_envs, nt, n, 3), dtype=torch.float64, device=dev)
        gT = torch.zeros((self.n_envs, nt, 3), dtype=torch.float64, device=dev)
        p = lambda t: t.data_ptr() if t is not None else None
        io = L.MpmAdjointIO(xbar=p(seeds[0]), vbar=p(seeds[1]), Cbar=p(seeds[2]), Fbar=p(seeds[3]),
                            xbar0=p(outs[0]), vbar0=p(outs[1]), Cbar0=p(outs[2]), Fbar0=p(outs[3]),
                            gE=p(gE), gnu=p(gnu), gu=p(gu) if self.max_tools else None,
                            gT=p(gT) if self.max_tools else None)
        L.check(self.lib.mpm_substep_adjoint(self.ctx, int(n), ct.byref(io), _stream_ptr(stream)), self.ctx)
        return dict(xbar0=outs[0], vbar0=outs[1], Cbar0=outs[2], Fbar0=outs[3], gE=gE, gnu=gnu,
                    gu=gu[:, :self.max_tools], gT=gT[:, :self.max_tools])

    def positions(self):
        """All particle positions, (Ntot, 3) device tensor, original order."""
        return torch.cat([self.read(L.F_X, e).T for e in range(self.n_envs)], 0)

    def velocities(self):
        return torch.cat([self.read(L.F_V, e).T for e in range(self.n_envs)], 0)

    def profile(self, enable=True):
        L.check(self.lib.mpm_profile(self.ctx, 1 if enable else 0), self.ctx)

    def profile_report(self):
        """{kernel name: (total ms, launches)} of the built-in event timer."""
        out, k = {}, 0
        while True:
            name, ms, n = ct.c_char_p(), ct.c_double(), ct.c_int64()
            rc = self.lib.mpm_profile_read(self.ctx, k, ct.byref(name), ct.byref(ms), ct.byref(n))
            if rc != L.MPM_OK:
                break
            if n.value:
                out[name.value.decode()] = (ms.value, n.value)
            k += 1
        return out

    # ------------------------------------------------------------------ surface
    def extract_surface(self, env=0, iso=None, max_tris=None, stream=None):
        """Tissue surface of one environment as a (T, 3, 3) float32 device
        tensor of triangle vertices (mpm_extract_surface).  iso defaults to
        half the material density.  Without max_tris the count is taken first
        (one synchronisation), then the triangles."""
        if iso is None:
            iso = 0.5 * float(self.material[env, 2])
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        if max_tris is None:
            L.check(self.lib.mpm_extract_surface(self.ctx, env, float(iso), None, 0, ct.c_void_p(count.data_ptr()),
                                                 _stream_ptr(stream)), self.ctx)
            max_tris = int(count.item())
        tris = torch.empty((max(1, int(max_tris)), 3, 3), dtype=torch.float32, device=self.device)
        L.check(self.lib.mpm_extract_surface(self.ctx, env, float(iso), ct.c_void_p(tris.data_ptr()), int(max_tris),
                                             ct.c_void_p(count.data_ptr()), _stream_ptr(stream)), self.ctx)
        return tris[:min(int(max_tris), int(count.item()))], int(count.item())

    # ------------------------------------------------------------------ reads
    _PCOMPS = {L.F_X: 3, L.F_V: 3, L.F_C: 9, L.F_F: 9}
    _GCOMPS = {L.F_GRID_M: 1, L.F_GRID_MV: 3, L.F_GRID_V: 3, L.F_DENSITY: 1}

    def read(self, field, env=0, device=True):
        """A field of one environment as a torch tensor ([comps][N] particles,
        [comps][n^3] grid), on the device unless device=False (numpy)."""
        if field in self._PCOMPS:
            shape = (self._PCOMPS[field], int(self.np[env]))
        elif field in self._GCOMPS:
            shape = (self._GCOMPS[field], int(self.gn[env]) ** 3)
        elif field == L.F_STATUS:
            out = np.zeros(1, np.uint32)
            L.check(self.lib.mpm_read_state(self.ctx, env, field, out.ctypes.data_as(ct.c_void_p), 4, 0,
                                            _stream_ptr()), self.ctx)
            return int(out[0])
        elif field == L.F_STEP:
            out = np.zeros(1, np.int32)
            L.check(self.lib.mpm_read_state(self.ctx, env, field, out.ctypes.data_as(ct.c_void_p), 4, 0,
                                            _stream_ptr()), self.ctx)
            return int(out[0])
        elif field == L.F_TOOL_T:
            out = np.zeros((max(1, self.max_tools), 3), np.float64)
            L.check(self.lib.mpm_read_state(self.ctx, env, field, out.ctypes.data_as(ct.c_void_p), out.nbytes, 0,
                                            _stream_ptr()), self.ctx)
            return out[:self.max_tools]
        else:
            raise ValueError(field)
        if device:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
            L.check(self.lib.mpm_read_state(self.ctx, env, field, ct.c_void_p(out.data_ptr()), out.numel() * 4, 1,
                                            _stream_ptr()), self.ctx)
            return out
        out = np.empty(shape, np.float32)
        L.check(self.lib.mpm_read_state(self.ctx, env, field, out.ctypes.data_as(ct.c_void_p), out.nbytes, 0,
                                        _stream_ptr()), self.ctx)
        return out

    def particles(self, env=0):
        """(x (N,3), v (N,3), C (N,3,3), F (N,3,3)) numpy float32, original order."""
        x = self.read(L.F_X, env, device=False).T
        v = self.read(L.F_V, env, device=False).T
        C = self.read(L.F_C, env, device=False).T.reshape(-1, 3, 3)
        F = self.read(L.F_F, env, device=False).T.reshape(-1, 3, 3)
        return x, v, C, F

    def grid(self, env=0):
        """(m (n,n,n), mv (n,n,n,3), v (n,n,n,3)) numpy float32."""
        n = int(self.gn[env])
        m = self.read(L.F_GRID_M, env, device=False).reshape(n, n, n)
        mv = self.read(L.F_GRID_MV, env, device=False).reshape(3, n, n, n).transpose(1, 2, 3, 0)
        v = self.read(L.F_GRID_V, env, device=False).reshape(3, n, n, n).transpose(1, 2, 3, 0)
        return m, mv, v

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            torch.cuda.synchronize()
            self.lib.mpm_destroy(self.ctx)
            self.ctx = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
