"""Seeded synthetic inputs for the recursive multiscale Robin coupled method.

This package only draws random fields and lays out boundary data.  It holds
none of the method's arithmetic, so both the CPU oracle and the GPU path can
take their inputs from it without sharing any of the computation.

Everything is deterministic given a seed (NumPy PCG64 ``default_rng``).
"""

from .fields import lognormal_grf, gaussian_field_exp, channelized, lognormal_grf3d  # noqa: F401
from .problems import (  # noqa: F401
    Problem,
    Problem3D,
    bc_faces3d,
    dirichlet_we3d,
    grf3d_problem,
    dirichlet_we,
    five_spot,
    config_problem,
    ensemble_member,
    CONFIGS,
)
