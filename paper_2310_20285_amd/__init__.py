"""IterNCGP hot path for AMD Instinct MI355X (gfx950).

The computation lives in the HIP library ``libitergp.so`` (C ABI in
``include/itergp.h``); :mod:`paper_2310_20285_amd.api` is a thin PyTorch-facing
binding of the same calls.  Importing this package does not load the library;
the first call does, and fails loudly when it is missing.
"""
__all__ = ["api", "build"]
