"""MI355X-native (gfx950, HIP, FP64) evolution of spherically symmetric scalar
collapse in AdS4 (Liebling & Khanna, arXiv:1706.07413), behind the ``adscl_*``
C-ABI library."""
