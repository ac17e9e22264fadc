"""MI355X library for the lattice-Boltzmann step of the reduced polyatomic
ES-BGK model (Kolluru, Atif & Ansumali, arXiv:2201.05280).

The step runs in hand-written HIP kernels (libpgk.so, C ABI in include/pgk.h);
`Solver` is a thin front end that takes device memory and streams from torch.
"""
from ._lib import (CN, DIRICHLET, E2, F3, F4, FP32DEV, FP64, LIT, PERIODIC, WALL, buffer_sizes,  # noqa: F401
                   load, resolve)
from .solver import Solver  # noqa: F401

THETA0 = 0.2948964908710633
