"""MI355X (gfx950) implementation of the SSsNAL method for the linear C-SVC
dual QP (arXiv 1910.01312): hand-written HIP kernels behind the C ABI in
include/ssnalm.h, with a thin Python front end.

    from paper_1910_01312_amd import Solver, solve
    x, w, info = solve(X, y, C, tol=1e-6)
"""
from __future__ import annotations

__all__ = ["Solver", "solve", "build"]


def __getattr__(name):
    if name in ("Solver", "solve"):
        from . import solver
        return getattr(solver, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
