"""MI355X-native (gfx950, HIP) multigrid solver for the NR99 linear
magnetohydrostatic potential, after MacTaggart et al. (arXiv:1307.6720).

The computation lives in libmhs.so (C ABI: include/mhs.h); this package
marshals torch tensors into it.  Importing the package does not load the
library; the first call does, and fails loudly if it has not been built.
"""

from ._lib import PLAN_GENERAL, PREC_FP64, PREC_MIXED, MHSError  # noqa: F401

__all__ = ["PREC_FP64", "PREC_MIXED", "PLAN_GENERAL", "MHSError", "Plan", "solve", "make_opts", "workspace_bytes"]


def __getattr__(name):
    if name in ("Plan", "solve", "make_opts", "workspace_bytes", "GridSpec", "SolveResult"):
        from . import solver

        return getattr(solver, name)
    raise AttributeError(name)
