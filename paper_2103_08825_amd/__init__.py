"""MI355X (gfx950) engine for iterated star and box stencil sweeps.

The computation is that of Li et al., "An Efficient Vectorization Scheme for
Stencil Computation" (arXiv 2103.08825), Section 1: T Jacobi steps in which
each point becomes a weighted sum of its order-r neighbourhood.  The engine is
the C-ABI library ``libstencil.so`` (header ``include/stencil.h``) built from
``csrc/``; this package holds its thin Python binding (``_lib``), torch-facing
wrappers (``api``), the autograd function (``autograd``) and seeded input
generators (``workloads``).  Importing the package loads nothing; the library
is loaded on first use and its absence is an error.
"""
__all__ = ["Plan", "offsets", "num_points", "reduce", "StencilFn", "run_batched", "Batch"]


def __getattr__(name):
    if name in ("Plan", "offsets", "num_points", "reduce"):
        from . import api
        return getattr(api, name)
    if name in ("StencilFn",):
        from . import autograd
        return getattr(autograd, name)
    if name in ("run_batched", "Batch"):
        from . import batched
        return getattr(batched, name)
    raise AttributeError(name)
