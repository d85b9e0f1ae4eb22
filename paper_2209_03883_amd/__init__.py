"""MI355X (gfx950) OFDM monostatic radar receive path.

The compute path is the HIP library libradar.so (C ABI in include/radar.h);
``radar`` is its Python binding.
"""
