"""MI355X (gfx950) implementation of the per-step NEP molecular-dynamics hot path.

Submodules:
  inputs  seeded synthetic workloads and random-weight models (no NEP arithmetic)
  nep     ctypes binding of libnep.so (the C-ABI in include/nep.h)
  build   compiles libnep.so in-tree with hipcc for gfx950
Importing the package loads nothing; ``nep`` loads the HIP library on first use.
"""
