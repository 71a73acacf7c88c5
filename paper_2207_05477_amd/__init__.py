"""MI355X (gfx950) Evoformer block: HIP kernels behind the C ABI of
include/evo.h (libevo.so), with a ctypes binding and autograd wrappers.

The product path has no CPU fallback: if libevo.so is missing, calls raise.
"""
from ._abi import EXPORTS, EvoError, LIB_PATH, load  # noqa: F401

__all__ = ["EXPORTS", "EvoError", "LIB_PATH", "load", "binding", "autograd"]


def __getattr__(name):
    if name in ("binding", "autograd"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
