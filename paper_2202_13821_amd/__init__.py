"""MI355X-native DG-HGKS: one S2O4 step of the modal DG gas-kinetic scheme
(arXiv 2202.13821) behind the C-ABI of include/dg_hgks.h, with hand-written
HIP kernels for gfx950.  torch supplies device memory and streams."""
from . import problems  # noqa: F401
from ._lib import DGHGKSError, load  # noqa: F401
from .solver import DGHGKSSteps, Solver, kinetic_energy, step_noalloc, steps, tgv_history  # noqa: F401
