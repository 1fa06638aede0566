"""MI355X (gfx950) relativistic lattice Boltzmann library for particles of
finite mass (arXiv:1703.04605): HIP kernels behind the C ABI of
include/rlbm.h, with a thin ctypes binding in ``rlbm``."""
from . import rlbm  # noqa: F401
