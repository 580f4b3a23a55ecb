"""MI355X voxel Monte Carlo engine for internal dosimetry (ARCHER-NM method,
arXiv 2111.11687): HIP kernels behind the C ABI of include/nmdose.h.

``binding`` holds the ctypes wrappers of the C entry points (the library is
loaded on first use; there is no CPU path), ``phantoms`` the seeded synthetic
inputs.
"""
from . import binding, phantoms  # noqa: F401

__all__ = ["binding", "phantoms"]
