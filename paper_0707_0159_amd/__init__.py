"""MI355X (gfx950) superblock Hv and Lanczos of the direct 2-D DMRG.

The compute path is the HIP library ``libd2d.so`` (C ABI in include/d2d.h);
``paper_0707_0159_amd.d2d`` is its Python binding.
"""
from . import d2d  # noqa: F401
