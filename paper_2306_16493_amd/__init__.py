"""MI355X (gfx950) electron-phonon Wannier interpolation SERTA transport path.

The computation lives in the HIP library ``libeph.so`` behind the C ABI of
``include/eph.h``; ``eph`` is its Python binding.
"""
from .eph import (  # noqa: F401
    Context, EphError, RatesParams, Counts, lib, LIB_PATH, EXPORTS, PRECISIONS, mobility,
)
