"""MI355X (gfx950) parallel multi-scale reduction of persistent-homology
boundary matrices over F2 (Mendoza-Smith & Tanner, arXiv 1708.04710).

The compute path is the HIP library ``libpms.so`` (C ABI in
``include/pms.h``); this package is its thin Python binding.  Importing the
package does not load the library; the first call does, and fails loudly if
it has not been built.
"""
from __future__ import annotations

__all__ = ["reduce", "default_options", "ReduceResult", "PmsError"]


def __getattr__(name):
    if name in ("reduce", "default_options", "ReduceResult"):
        from . import api
        return getattr(api, name)
    if name == "PmsError":
        from ._binding import PmsError
        return PmsError
    raise AttributeError(name)
