"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds geometry and initial-field generators only. It contains none
of the lattice Boltzmann arithmetic, none of the enumeration / adjacency / run
logic and no lattice constants, so the oracle and the HIP path stay
independent of each other while consuming identical inputs.

Masks are ``uint8`` arrays of shape ``(nx, ny, nz)`` in C order (x slowest,
z fastest); a nonzero entry marks a solid voxel.
"""

from .geometry import (  # noqa: F401
    channel_mask,
    rsa_spheres,
    relaxed_spheres,
    foam,
    init_fields,
    pbb_fraction,
    workload,
    WORKLOADS,
)
