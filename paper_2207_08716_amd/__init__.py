"""MI355X (gfx950) pseudo-transient solver for 3D poro-visco-elastic
two-phase flow (thesis article 1, section 2.2).

The computation runs in hand-written HIP kernels behind the C ABI of
include/ptporo.h (libptporo.so, built in-tree by ``build.build()``).  Python
supplies device memory and streams through torch and marshals arguments.
"""
from . import inputs, teff  # noqa: F401

__all__ = ["inputs", "teff", "Grid", "schedules"]


def __getattr__(name):
    # the GPU handle needs the built library and torch; import lazily
    import importlib
    if name == "Grid":
        return importlib.import_module(".grid", __name__).Grid
    if name in ("schedules", "grid", "abi", "build"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
