"""MI355X-native diffuse-solid ternary lattice Boltzmann step (arXiv 2504.19941).

The step runs in hand-written HIP kernels for gfx950 behind the C ABI of
``libdsm.so`` (declared in include/dsm.h); :mod:`.dsm` is the thin Python
binding over that ABI.  :mod:`.workloads` generates seeded synthetic inputs
and :mod:`.analysis` measures contact angles from fields.
"""
