"""MI355X-native DNN-MG fine-level correction (arXiv 2307.14837).

The compute lives in libdnnmg.so (hand-written HIP for gfx950 behind the C ABI
declared in include/dnnmg.h).  ``_lib`` is the thin ctypes binding with the
same entry-point names; ``stepper`` strings the calls into one correction
step.  Importing the binding fails loudly when the library is not built.
"""
from . import _lib  # noqa: F401
from ._lib import *  # noqa: F401,F403

__all__ = list(_lib.EXPORTS)
