"""MI355X-native immersed-boundary lattice Boltzmann solver (D3Q19 BGK with
Guo forcing + implicit velocity-correction IBM), after Kumar, De & Das,
"Investigation of flow field of clap & fling motion using immersed boundary
coupled lattice Boltzmann method".

The solver is the C-ABI library libibmlbm.so (include/ibmlbm.h) built from
csrc/ for gfx950; `Solver` is a thin ctypes binding over it.
"""
from .solver import Solver, complete_case, lattice_params  # noqa: F401
