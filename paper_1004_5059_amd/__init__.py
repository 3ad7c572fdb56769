"""MI355X-native thermal volumetric lattice Boltzmann (TVLBM) hot path.

The computation lives in hand-written HIP kernels for gfx950 behind the C ABI
of include/tvlbm.h (``_lib/libtvlbm.so``); ``tvlbm`` is the Python binding.
"""
