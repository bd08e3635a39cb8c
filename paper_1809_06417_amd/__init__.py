"""MI355X (gfx950) implementation of the hot path of radiative-transport
flame volume reconstruction (Shen et al., arXiv:1809.06417).

The compute lives in librte.so (HIP kernels behind the C ABI of
include/rte.h); :mod:`paper_1809_06417_amd.rte` is its thin Python binding.
Importing this package does not load the library; the binding loads it on
first use and raises if it has not been built.
"""
__version__ = "0.1.0"
