"""MI355X-native differentiable AMG-PCG (smoothed aggregation) on CSR.

The solve path runs in hand-written HIP kernels for gfx950 behind a C ABI
(``include/amg355.h``); this package is its thin Python binding.
"""
