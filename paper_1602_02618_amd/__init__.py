"""MI355X-native Chebyshev--Jacobi transform (forward and inverse) on HIP.

The transform itself lives in the HIP library that `csrc/` builds
(`libcjt_hip.so`, C-ABI declared in `include/cjt.h`); `cjt.py` is the thin
ctypes binding with the same names.  Importing this package loads nothing;
the library is opened on first use and an error is raised if it is missing.
"""
import importlib

__all__ = ["cjt", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
