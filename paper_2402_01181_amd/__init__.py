"""MLS-MPM Neo-Hookean tissue substep (arXiv 2402.01181, Sec. III-B/III-C)
on AMD MI355X: hand-written HIP kernels for gfx950 behind a C ABI
(include/mpm.h), with a thin Python binding.

``scenes`` (seeded inputs) imports without a GPU; ``Sim`` needs the built
library and a ROCm device and has no CPU fallback.
"""
from . import scenes  # noqa: F401


def __getattr__(name):
    if name in ("Sim",):
        from .sim import Sim
        return Sim
    raise AttributeError(name)
