"""Seeded synthetic inputs for the spectral boundary-integral (SBI) wave solver.

This package is shared by the FP64 CPU oracle and the GPU path.  It only builds
input fields (sea states, bathymetries, steady-wave initial conditions) and holds
none of the solver's arithmetic: no Fourier multipliers of the method, no
vertical-velocity expansion, no time stepping.
"""
from .generators import (  # noqa: F401
    GridSpec,
    jonswap_crossing_sea,
    stokes2_finite_depth,
    stokes3_deep,
    gaussian_bump_depth,
    trapezoid_bar_depth,
    undulating_bars_depth,
    random_bumps_depth,
    band_limited_random,
    narrowband_random,
    config_c1,
    config_c2,
    config_c3,
    config_c4_member,
    config_c5,
)
