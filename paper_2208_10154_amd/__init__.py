"""Batched HEALPix spherical harmonic transforms on AMD MI355X (gfx950).

The transforms run in ``libsht.so`` (hand-written HIP kernels behind a C ABI,
``include/sht.h``); :mod:`paper_2208_10154_amd.sht` is its ctypes binding and
:mod:`paper_2208_10154_amd.serve` the batching request loop on top of it.
"""
