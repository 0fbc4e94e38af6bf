"""Sparse-lattice D3Q19 lattice Boltzmann propagation steps for MI355X.

Hot path of Wittmann, Zeiser, Hager and Wellein (arXiv:1410.0412): fused
BGK collide-and-propagate steps over a fluid-only node list with an indirect
adjacency list, as two-grid OS-NT or one-grid AA pattern, each with plain or
reduced indirect addressing (RIA). All work runs in ``liblbm_sparse.so``
(C++ lattice builder, HIP kernels for gfx950); this package only marshals
arguments.
"""

from ._capi import LbmError, lib  # noqa: F401
from .lattice import Lattice  # noqa: F401
from .solver import Solver, bench_stream, choose_index, choose_odd_schedule, required_bytes  # noqa: F401
from .adjoint import OutletFlux, outlet_flux  # noqa: F401
