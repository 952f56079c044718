"""MI355X-native speculative progressive isosurface raycasting (arXiv 2309.10212).

The product is the C-ABI shared library ``libspr.so`` (HIP, gfx950) declared in
``include/spr.h``; :mod:`paper_2309_10212_amd.spr` is its ctypes binding.
"""
from .spr import (Batch, Camera, Context, PassStats, Render, SprError, Volume, load_library,  # noqa: F401
                  version, HIT_DTYPE, NONE, DTYPE_F32, DTYPE_U8)
