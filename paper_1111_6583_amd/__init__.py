"""MI355X-native finite-volume step library (PyClaw method, arXiv 1111.6583).

The compute path is ``libclaw.so`` (hand-written HIP for gfx950 behind a C
ABI, ``include/claw.h``); this package only marshals arguments to it.
Importing the package does not load the library; ``Solver`` does, and fails
loudly when it is missing.
"""

__all__ = ["Solver", "Batch", "load_library"]


def __getattr__(name):
    if name in ("Solver", "Batch"):
        from . import solver
        return getattr(solver, name)
    if name == "load_library":
        from ._claw import load_library
        return load_library
    raise AttributeError(name)
