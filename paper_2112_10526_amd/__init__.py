"""MI355X-native hot path of RBM variational Monte Carlo (NetKet 3 paper,
arXiv 2112.10526): hand-written CDNA4 HIP kernels behind the C ABI of
``libnqs.so`` (include/nqs.h), with a thin Python binding.

Importing the package does not touch the GPU; constructing a ``VMCState``
loads ``libnqs.so`` and fails loudly if it or the device is missing.
"""
from . import _lib  # noqa: F401

__all__ = ["VMCState", "batch_step", "load_library"]


def load_library():
    return _lib.load()


def __getattr__(name):
    if name in ("VMCState", "batch_step"):
        from . import nqs
        return getattr(nqs, name)
    raise AttributeError(name)
