"""MI355X (gfx950) implementation of the sub-grid-bathymetry DG shallow-water
operator of arXiv:2505.18743: HIP kernels behind the C ABI in include/sw.h,
with a thin ctypes binding (``binding.Solver``)."""
from .binding import Ensemble, Solver, load, EXPORTS  # noqa: F401
