"""MI355X-native D3Q19 lattice-Boltzmann + immersed-boundary hot path (gfx950 HIP).

The compute lives in the C-ABI library ``liblbmib.so`` built from ``csrc/``; the
Python layer (``lbm.py``) only marshals arguments into it.  Nothing is loaded at
import time, so the geometry generators in ``inputs`` can be used without a GPU.
"""
__all__ = ["inputs"]
