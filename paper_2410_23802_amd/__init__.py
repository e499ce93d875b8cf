"""MI355X-native volumetric lattice Boltzmann solver for particle-resolved
thermal particulate flow with conjugate heat transfer (arXiv 2410.23802).

The solver is the HIP library libvlb.so (C ABI in include/vlb.h); `vlb` is
its Python binding.  Build with `paper_2410_23802_amd.build.build()`.
"""
from . import vlb  # noqa: F401
from .vlb import Domain, VlbError, VlbLibraryMissing  # noqa: F401
