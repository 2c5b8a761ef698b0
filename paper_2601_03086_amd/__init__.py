"""MI355X-native finite-element physics path of the Pretrained Finite Element
Method (arXiv 2601.03086): P1 energy / internal force / Hessian-vector
kernels, warm-started Jacobi-PCG and Newton-Krylov solves, a batched
differentiable energy and a continuous-batching solve server.

The compute lives in libpfem.so (hand-written HIP for gfx950) behind the C
ABI in include/pfem.h.  This package is its thin Python binding.
"""
from ._lib import PfemError, load  # noqa: F401

__all__ = ["PfemError", "load", "core", "autograd"]


def __getattr__(name):
    if name in ("core", "autograd"):
        import importlib
        return importlib.import_module("." + name, __name__)
    if name in ("Context", "Mesh", "Batch", "Server"):
        from . import core
        return getattr(core, name)
    raise AttributeError(name)
