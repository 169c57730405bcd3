"""MI355X-native range analysis of MLP implicit surfaces (affine arithmetic
bounds, classification, octree subdivision, ray casting) after Sharp &
Jacobson, "Spelunking the Deep" (ACM TOG 2022).

The computation lives in the HIP library ``libspk.so`` (C ABI in
``include/spk.h``); :mod:`paper_2202_02444_amd.spk` is its Python binding.
"""
from . import spk  # noqa: F401

__all__ = ["spk"]
