"""MI355X (gfx950) coupled lattice-Boltzmann / bead-dynamics hot path (arXiv:0710.1272).

The compute path is the HIP library liblbmd.so (C ABI in include/lbmd.h); this
package only marshals arguments to it (paper_0710_1272_amd.lbmd).
"""
from . import lbmd  # noqa: F401
from .lbmd import Simulation  # noqa: F401
