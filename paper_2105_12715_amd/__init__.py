"""Restarted PDHG for linear programs on MI355X (gfx950).

The solver lives in the HIP library ``libpdhg.so`` behind the C ABI of
``include/pdhg.h``; ``_lib`` is its ctypes binding.  ``lpgen`` draws the
seeded planted-optimum workloads.  Importing the package loads nothing;
the library is opened on first use.
"""
import importlib

from . import lpgen  # noqa: F401


def __getattr__(name):
    if name.startswith("__") or name == "_lib":
        raise AttributeError(name)
    lib = importlib.import_module(__name__ + "._lib")
    if hasattr(lib, name):
        return getattr(lib, name)
    raise AttributeError(name)
