"""MI355X-native homogenized lattice Boltzmann (HLBM) sweep.

The compute path is the C-ABI library ``libhlbm.so`` (hand-written HIP for
gfx950) declared in ``include/hlbm.h``; :mod:`paper_2310_14746_amd.hlbm` is its
thin ctypes binding.  Importing this package does not load the library, so the
input generators in :mod:`paper_2310_14746_amd.inputs` can be used on their own.
"""
