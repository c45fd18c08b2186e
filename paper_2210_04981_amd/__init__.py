"""MI355X-native hybrid depth of field (Tan et al., SIGGRAPH 2020 posters).

The product is ``libhdof.so`` (HIP for gfx950 behind the C ABI in
``include/hdof.h``); ``paper_2210_04981_amd.hdof`` is its Python binding.
Build with ``python -m paper_2210_04981_amd.build``.
"""
__all__ = ["hdof", "build"]
