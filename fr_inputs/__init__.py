"""Seeded synthetic inputs shared by the FR library tests, the bench and the oracle.

This package only *describes* problems: mesh node coordinates and connectivity,
boundary tags, analytic initial fields and seeded noise.  It contains none of the
flux-reconstruction arithmetic (no solution/flux points, no operators, no
fluxes); both the oracle and the HIP path compute those on their own.
"""
from .meshes import (  # noqa: F401
    FACE_AUTO, BC_WALL, BC_FARFIELD,
    MeshDesc, gll_points, periodic_box, o_grid, cavity, c_grid_naca, concat_meshes, sponge_degrees,
)
from .fields import (  # noqa: F401
    FlowParams, freestream_params, vortex_params, vortex_state, freestream_state,
    entropy_wave_state, shear_wave_state, thermal_wave_state, noise_like, developed_state,
)
