"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds only the problem specification: configuration numbers,
voxelised material maps, model curves sampled on the radial grid (potentials,
transition dipole, initial wavefunction) and incident-pulse samples.  It holds
none of the propagation arithmetic; both the oracle and the HIP library take
what it produces as inputs.
"""

from .configs import CONFIGS, Config, get_config  # noqa: F401
