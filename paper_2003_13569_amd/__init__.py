"""MI355X-native fractional ETDRK4 (Almushaira and Bhatt): libsfrde and its
Python binding.

``sfrde``      ctypes binding of the C ABI (include/sfrde.h), same names.
``torch_api``  Plan bound to torch tensors and streams; SFRDEFunction.
``build``      compiles csrc/ into libsfrde.so for gfx950.
"""
from . import sfrde  # noqa: F401

__all__ = ["sfrde"]
