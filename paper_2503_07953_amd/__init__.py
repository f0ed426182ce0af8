"""MI355X-native right-hand side of the five-equation diffuse-interface model.

The package holds the HIP library (``libmfc355.so``, sources in ``csrc/``,
C ABI in ``include/mfc355.h``) and its thin Python binding:

* ``Solver`` -- one library context; prim/cons conversion, RHS, SSP-RK3 step,
  signal speed, conservation sums, non-finite check.
* ``build()`` -- compile the library for gfx950 in-tree.
"""
from .builder import build  # noqa: F401
from ._lib import MfcError, LibraryMissing, load  # noqa: F401


def __getattr__(name):
    # torch-dependent front ends are imported lazily
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name in ("autograd",):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
