"""MI355X-native matrix-free photoacoustic operator A and its adjoint A^T.

The operator and its C ABI live in ``libpatop.so`` (HIP, gfx950), built from
``csrc/`` by ``build.py``.  ``_lib`` is the ctypes binding and ``operator``
the torch wrapper (device memory, streams, autograd)."""
from . import _lib  # noqa: F401

__all__ = ["_lib", "operator"]
