"""MI355X (gfx950) causal-set generator and Benincasa-Dowker action library.

After W. J. Cunningham and D. Krioukov, "Causal Set Generator and Action
Computer", arXiv:1709.03013.  The computation lives in ``libcs_gfx950.so``
(HIP kernels + C ABI, ``include/cs.h``); this package is a thin ctypes
binding with the same function names.  Build with
``python -m paper_1709_03013_amd.build``.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import BatchCall, CsError, lib, exported_symbols  # noqa: F401

__all__ = [n for n in dir() if n.startswith("cs_")] + ["BatchCall", "CsError", "lib", "exported_symbols"]
