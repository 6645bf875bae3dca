"""A-orthonormalising modified Gram-Schmidt (naive / HA / HP) on MI355X.

The compute path is the HIP library ``libamgs.so`` reached through a C ABI
(``include/amgs.h``); ``paper_1703_10440_amd.amgs`` is its thin ctypes
binding.  Importing this package loads nothing: the library is loaded on
first use, and a missing library raises instead of falling back to anything.
"""

__all__ = ["inputs", "amgs"]
