"""Seeded synthetic workloads for Bluebild standard synthesis.

This package builds the *inputs* of the imaging problem: antenna layouts,
pixel grids, skies, visibility matrices and energy-level partitions.  It
simulates the instrument (the measurement model of Section 2.1) but holds none
of the imaging arithmetic (Gram matrix, eigensolve, phase synthesis, level
reduction); both the FP64 oracle and the GPU library consume what it returns.

Every random draw comes from ``rng(config_id, stream_id)`` so that any
instance can be rebuilt from its config id and index alone.
"""

from .seeds import rng, SEED_BASE  # noqa: F401
from .geometry import (  # noqa: F401
    C_LIGHT,
    wavelength_m,
    disk_layout,
    spiral_layout,
    enu_to_ecef,
    earth_rotate,
    hour_angles,
    pixel_grid,
    pixel_index_direction,
    tangent_basis,
)
from .sky import point_sources, gaussian_blobs, grid_sources  # noqa: F401
from .visibilities import (  # noqa: F401
    steering,
    visibility,
    hermitian_noise,
    psd_noise,
    add_noise_snr,
)
from .levels import kmeans1d_intervals, levels_from_intervals  # noqa: F401
from .random_fields import random_eigvecs, random_eigvals  # noqa: F401
from .sampling import sample_pixels  # noqa: F401
from . import configs  # noqa: F401
