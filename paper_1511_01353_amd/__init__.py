"""MI355X-native free-mesh transform (octree-scoped polynomial interpolant).

The work runs in libfmt.so (HIP kernels for gfx950 behind the C ABI of
include/fmt.h); this package is its Python binding.
"""
from .fmt import *  # noqa: F401,F403
from .fmt import EXPORTED, Tree, FmtError, load_library, LIB_PATH  # noqa: F401

__all__ = [n for n in dir() if n.startswith("fmt_") or n.startswith("FMT_")] + [
    "Tree", "FmtError", "load_library", "LIB_PATH"]
