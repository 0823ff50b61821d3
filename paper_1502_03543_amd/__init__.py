"""MI355X (gfx950) Primal-Dual Affine Scaling: the per-iteration Newton solve
(normal matrix, Cholesky, triangular solves, direction, ratio test, step) as
hand-written HIP kernels behind a C ABI (include/pdas.h), with a thin Python
binding.  See Divakar, "Primal Dual Affine Scaling on GPUs", arXiv 1502.03543.
"""
from . import capi  # noqa: F401
from . import lpgen  # noqa: F401

__all__ = ["capi", "lpgen", "solver"]


def __getattr__(name):
    # torch is imported lazily so that the C-ABI checks run without it
    if name == "solver":
        import importlib
        return importlib.import_module(__name__ + ".solver")
    raise AttributeError(name)
