"""Flexibly enlarged Conjugate Gradient on MI355X (gfx950).

The solver lives in the HIP library ``libecg.so`` (C ABI: ``include/ecg.h``);
``paper_2305_19013_amd.ecg`` is its Python binding.  Importing the package does
not touch the GPU; calling into the binding requires the built library.
"""

from . import ecg  # noqa: F401

__all__ = ["ecg"]
