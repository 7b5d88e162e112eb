"""MI355X-native out-of-core stencil computation with on-the-fly fixed-rate
compression (Shen, Wu, Okita, Ino, arXiv 2109.05410).

The computation lives in liboocs.so (HIP for gfx950, C ABI in
include/oocs.h); `api` is the Python binding. Importing this package does not
load the library; the first call into `api` does, and fails loudly if the
library has not been built.
"""
import importlib

__all__ = ["api", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
