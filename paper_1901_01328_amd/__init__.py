"""KPA grouping path of StreamBox-HBM on AMD MI355X (gfx950).

The compute lives in libkpa.so (hand-written HIP kernels behind a C ABI,
declared in include/kpa.h); ``kpa`` is its ctypes binding.  Import of the
binding fails if the library has not been built.
"""
import os as _os

LIB_PATH = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "libkpa.so")


def load():
    """Import and return the binding module (raises ImportError if unbuilt)."""
    from . import kpa
    return kpa
