"""MI355X-native moment-chain lattice Boltzmann method for hyperelastic solids.

The time step runs in hand-written HIP kernels for gfx950 behind a small C ABI
(``include/mclbm.h``); ``mclbm`` is the thin Python binding of that ABI and
``workloads`` describes seeded synthetic problems.  Importing the package does
not load the native library; ``paper_2502_00920_amd.mclbm`` does.
"""
__all__ = ["mclbm", "workloads"]
