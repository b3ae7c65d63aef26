"""MI355X-native TrackerSplat motion transfer (libtg + Python binding).

The library is `libtg.so` (hand-written HIP for gfx950) behind the C ABI in
include/tg.h; this package marshals torch tensors into it.  Importing the
package does not load the library; the first call does, and raises if it has
not been built (there is no CPU fallback).
"""
from ._lib import TGError, lib  # noqa: F401

__version__ = "0.1.0"


def __getattr__(name):
    if name in ("api",):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    from . import api
    return getattr(api, name)
