"""Batched rigid-body kinematics and dynamics on MI355X (gfx950).

``Model`` and the operators live in :mod:`paper_2605_31481_amd.bard`, a thin
ctypes binding of ``libbard.so``; :func:`paper_2605_31481_amd.build.build`
compiles that library.  The binding is loaded on first attribute access so the
build step can run before the library exists.
"""

import importlib

__all__ = ["Model", "BardError", "as_batch_major", "WORLD", "LOCAL_WORLD_ALIGNED"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".bard"), name)
    raise AttributeError(name)
