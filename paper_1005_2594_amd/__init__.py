"""MI355X-native time step of the coarse-grained blood model of Janoschek,
Toschi & Harting (arXiv:1005.2594): D3Q19 lattice-Boltzmann plasma coupled to
rigid ellipsoidal cells, as hand-written HIP for gfx950 behind a C ABI
(``include/cgb.h``).  ``paper_1005_2594_amd.cgb`` is the Python binding.
"""
from .cgb import (Batch, CgbError, Mlp, Sim, lib, P64, P32, PMX16, PMXBF16, PRECISIONS)  # noqa: F401
