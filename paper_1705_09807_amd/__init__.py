"""MI355X (gfx950) engine for the filtered large-eddy lattice-Boltzmann MHD
method of Flint & Vahala (arXiv 1705.09807).

The method runs in hand-written HIP kernels behind the C ABI of
include/lbmhd.h (liblbmhd.so); this package only builds and binds it.
"""

from .sim import Sim, make_params  # noqa: F401
