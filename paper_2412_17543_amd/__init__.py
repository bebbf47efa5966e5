"""MI355X (gfx950) deflated PCG with three-level BDDC and Krylov subspace recycling.

Hot path in hand-written HIP behind the C ABI of ``include/bddc.h``;
``Solver`` and ``DPCGSolveFn`` are thin wrappers (marshalling only).
"""
from ._lib import BddcError, load  # noqa: F401


def __getattr__(name):
    if name in ("Solver", "DPCGSolveFn"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
