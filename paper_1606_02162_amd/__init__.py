"""MI355X-native k-hop Fruchterman-Reingold layout (GiLA's hot path).

The compute path is the HIP library ``libgila.so`` (hand-written gfx950
kernels behind a C ABI, declared in ``include/gila.h``); ``gila`` is its thin
ctypes binding.  ``inputs`` holds the seeded synthetic input generators.
"""
