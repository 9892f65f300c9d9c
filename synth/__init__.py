"""Seeded synthetic inputs shared by the HIP path, the CPU oracle, the tests and the bench.

This package only *prepares inputs*: grid descriptions, boundary-condition kinds,
fluid and model parameters, and the solid indicator field lambda of each
workload.  It performs none of the solver's arithmetic (no discretisation, no
interpolation, no wall function, no linear algebra), so both implementations can
consume it without sharing any part of the method itself.
"""

from .cases import (  # noqa: F401
    CaseSpec,
    DEFAULT_CONSTANTS,
    case_bfs,
    case_ahmed,
    case_ahmed_small,
    case_channel_ib,
    case_channel_bodyfitted,
    case_cavity_block,
    case_small_body3d,
    case_uniform_duct,
    case_naca,
    naca_sweep_specs,
    case_bend2d,
)
from .geometry import (  # noqa: F401
    lambda_from_sdf,
    sdf_box,
    sdf_ahmed_like,
    sdf_halfspace,
    sdf_sphere,
    sdf_naca_symmetric,
    sdf_lbend,
    naca4_half_thickness,
)
