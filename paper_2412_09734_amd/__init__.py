"""MI355X-native restarted Halpern PDHG (r2HPDHG) for LP behind a C ABI.

`Solver` wraps libpdhg (include/pdhg.h); `build()` compiles the HIP library
for gfx950 in-tree.
"""

from ._build import build, LIB  # noqa: F401

__all__ = ["build", "LIB", "Solver", "options"]


def __getattr__(name):
    # torch is imported lazily so that building needs no GPU stack
    if name in ("Solver", "options"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
