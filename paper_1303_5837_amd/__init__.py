"""Multilevel (tree) Householder QR on one MI355X: TSQR panels and CAQR.

The compute path is the HIP library ``libcaqr.so`` (C ABI, declared in
``include/caqr.h``); :mod:`paper_1303_5837_amd.caqr` is its thin ctypes binding.
Importing this package does not load the library; the first call into
:mod:`~paper_1303_5837_amd.caqr` does, and fails loudly when it is missing.
"""
__all__ = ["inputs", "caqr"]
