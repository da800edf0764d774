"""PRISM (arxiv 2604.00250) analysis-by-synthesis pass on MI355X.

The per-iteration fused forward + adjoint pass, its priors, reductions and
optimiser steps run in hand-written HIP kernels for gfx950 inside
``libprism.so`` (C ABI in ``include/prism.h``); this package is the thin
binding (``_lib``, ``problem``), the autograd wrapper (``autograd``), the
graph-captured fit loop (``fit``), the launch autotuner (``tune``) and the
seeded synthetic workloads (``inputs``).
"""
from . import inputs  # noqa: F401  (pure NumPy, importable everywhere)

__all__ = ["inputs", "build", "lib", "Problem", "DeviceState"]


def build(verbose: bool = False) -> str:
    from .build import build as _b
    return _b(verbose)


def lib():
    from ._lib import lib as _l
    return _l()


def __getattr__(name):
    if name in ("Problem", "DeviceState", "adam_step_ptr", "rprop_step_ptr"):
        from . import problem
        return getattr(problem, name)
    raise AttributeError(name)
