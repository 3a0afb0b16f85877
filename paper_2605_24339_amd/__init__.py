"""MI355X-native GMCP hot path (Geometric Mortar Contact Potential).

The kernels live in ``libgmcp.so`` (HIP, gfx950) behind the C ABI declared in
``include/gmcp.h``; :class:`Context` marshals torch tensors to it.
"""
from ._native import NativeMissing  # noqa: F401


def __getattr__(name):
    # torch-dependent front end, imported lazily so the C-ABI checks run without it
    if name in ("Context", "GMCPError", "BSR", "Assembly"):
        from . import gmcp
        return getattr(gmcp, name)
    raise AttributeError(name)
