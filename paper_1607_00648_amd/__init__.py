"""MI355X (gfx950) quasi-matrix-free hybrid multigrid (arXiv:1607.00648).

The solver lives in the HIP library ``libqmg.so`` behind the C ABI of
``include/qmg.h``; ``qmg`` is its ctypes binding.  Importing this package does
not load the library; ``qmg.load()`` does, and raises if it is missing.
"""
from . import qmg  # noqa: F401

__all__ = ["qmg"]
