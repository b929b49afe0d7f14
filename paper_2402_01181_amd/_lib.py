"""ctypes binding of ``libmpm355.so`` (the C ABI declared in include/mpm.h).

Argument marshalling only: every step of the substep runs in the library's
HIP kernels.  The library is loaded after torch so both share torch's HIP
runtime.  There is no fallback: a missing library or GPU raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmpm355.so")

MPM_OK, MPM_E_ARG, MPM_E_HIP, MPM_E_STATE, MPM_E_UNSUPPORTED, MPM_E_WORKSPACE = 0, -1, -2, -3, -4, -5
FLAG_OUT_OF_DOMAIN, FLAG_INVERTED, FLAG_NONFINITE, FLAG_BARRIER_TIMEOUT = 1, 2, 4, 8
F_X, F_V, F_C, F_F, F_GRID_M, F_GRID_MV, F_GRID_V, F_STATUS, F_TOOL_T, F_STEP, F_DENSITY = range(11)
TOOL_CAPSULE, TOOL_BOX, TOOL_SDF = 0, 1, 2
SDF_NEAREST, SDF_TRILINEAR = 0, 1
CONTACT_SLIP, CONTACT_STICKY = 0, 1
STAGE_P2G, STAGE_GRID, STAGE_G2P = 0, 1, 2
STAGE_TILED_P2G, STAGE_TILED_GRID, STAGE_TILED_FUSED, STAGE_TILED_FUSED_FULL, STAGE_TILED_G2P = 3, 4, 5, 6, 7
(OPT_SCHEME, OPT_SORT_EVERY, OPT_BLOCK, OPT_GRAPH, OPT_PERSISTENT, OPT_SPIN_LIMIT, OPT_ITEM, OPT_NODE_SLOTS,
 OPT_GRID_AT_STAGING) = range(9)
SCHEME_DIRECT, SCHEME_TILED = 0, 1
STATIC_WORKSPACE_BYTES = 64 << 20   # MPM_STATIC_WORKSPACE_BYTES: the workspace of mpm_create_static
# option values a new context starts with
OPT_DEFAULTS = {OPT_SCHEME: SCHEME_TILED, OPT_SORT_EVERY: 16, OPT_BLOCK: 256, OPT_GRAPH: 0, OPT_PERSISTENT: 0,
                OPT_ITEM: 512, OPT_NODE_SLOTS: 3, OPT_GRID_AT_STAGING: 0}

EXPORTS = ["mpm_workspace_size", "mpm_create", "mpm_create_static", "mpm_destroy", "mpm_set_tool", "mpm_set_option",
           "mpm_substep", "mpm_run_stage", "mpm_substep_adjoint", "mpm_read_state", "mpm_last_error",
           "mpm_profile", "mpm_profile_read", "mpm_extract_surface"]


class MpmDesc(ct.Structure):
    _fields_ = [("n_envs", ct.c_int32), ("n_particles", ct.POINTER(ct.c_int32)),
                ("grid_n", ct.POINTER(ct.c_int32)), ("dt", ct.c_float), ("gravity", ct.c_float * 3),
                ("bound", ct.c_int32), ("max_tools", ct.c_int32), ("checkpoint_every", ct.c_int32),
                ("max_tape_substeps", ct.c_int32),
                ("x0", ct.c_void_p), ("v0", ct.c_void_p), ("C0", ct.c_void_p), ("F0", ct.c_void_p),
                ("material", ct.c_void_p), ("hold_tape", ct.c_int32)]


class MpmTool(ct.Structure):
    _fields_ = [("shape", ct.c_int32), ("contact", ct.c_int32), ("radius", ct.c_float),
                ("half_len", ct.c_float), ("friction", ct.c_float), ("theta", ct.c_float),
                ("R", ct.c_float * 9), ("T0", ct.c_float * 3), ("half", ct.c_float * 3),
                ("sdf_res", ct.c_int32), ("sdf_interp", ct.c_int32), ("sdf_h", ct.c_float),
                ("sdf_lo", ct.c_float * 3), ("sdf", ct.c_void_p)]


class MpmAdjointIO(ct.Structure):
    _fields_ = [("xbar", ct.c_void_p), ("vbar", ct.c_void_p), ("Cbar", ct.c_void_p), ("Fbar", ct.c_void_p),
                ("xbar0", ct.c_void_p), ("vbar0", ct.c_void_p), ("Cbar0", ct.c_void_p), ("Fbar0", ct.c_void_p),
                ("gE", ct.c_void_p), ("gnu", ct.c_void_p), ("gu", ct.c_void_p), ("gT", ct.c_void_p)]


class MpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mpm error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2402_01181_amd/build.py "
                          "(there is no CPU fallback)")
    L = ct.CDLL(path)
    vp, i32 = ct.c_void_p, ct.c_int32
    L.mpm_workspace_size.argtypes = [ct.POINTER(MpmDesc)]
    L.mpm_workspace_size.restype = ct.c_size_t
    L.mpm_create.argtypes = [ct.POINTER(MpmDesc), vp, ct.c_size_t, vp, ct.POINTER(vp)]
    L.mpm_create.restype = i32
    L.mpm_create_static.argtypes = [ct.POINTER(MpmDesc), vp, ct.POINTER(vp)]
    L.mpm_create_static.restype = i32
    L.mpm_destroy.argtypes = [vp]
    L.mpm_destroy.restype = None
    L.mpm_set_tool.argtypes = [vp, i32, i32, ct.POINTER(MpmTool), vp, i32]
    L.mpm_set_tool.restype = i32
    L.mpm_set_option.argtypes = [vp, i32, i32]
    L.mpm_set_option.restype = i32
    L.mpm_substep.argtypes = [vp, i32, i32, vp]
    L.mpm_substep.restype = i32
    L.mpm_run_stage.argtypes = [vp, i32, vp]
    L.mpm_run_stage.restype = i32
    L.mpm_substep_adjoint.argtypes = [vp, i32, ct.POINTER(MpmAdjointIO), vp]
    L.mpm_substep_adjoint.restype = i32
    L.mpm_read_state.argtypes = [vp, i32, i32, vp, ct.c_size_t, i32, vp]
    L.mpm_read_state.restype = i32
    L.mpm_extract_surface.argtypes = [vp, i32, ct.c_float, vp, ct.c_int64, vp, vp]
    L.mpm_extract_surface.restype = i32
    L.mpm_profile.argtypes = [vp, i32]
    L.mpm_profile.restype = i32
    L.mpm_profile_read.argtypes = [vp, i32, ct.POINTER(ct.c_char_p), ct.POINTER(ct.c_double),
                                   ct.POINTER(ct.c_int64)]
    L.mpm_profile_read.restype = i32
    L.mpm_last_error.argtypes = [vp]
    L.mpm_last_error.restype = ct.c_char_p
    _lib = L
    return L


def check(code, ctx=None):
    if code != MPM_OK:
        msg = load().mpm_last_error(ctx).decode()
        raise MpmError(code, msg)
    return code
