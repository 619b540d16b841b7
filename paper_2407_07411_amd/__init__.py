"""MI355X (gfx950) two-site DMRG effective-Hamiltonian library.

The compute lives in the HIP library `libdmrg_heff.so` (C ABI in
include/dmrg_heff.h); `paper_2407_07411_amd.heff` is its Python binding.
"""

__all__ = ["heff", "build"]
