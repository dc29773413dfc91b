"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input synthesis only (random fields, particle loads,
parameter draws).  It contains none of the gravity step's arithmetic, so
both the CPU oracle and the GPU path can take their inputs from it without
sharing any of the method's code.
"""
from .ics import (  # noqa: F401
    expected_variance,
    gaussian_field,
    lattice_displacement_ics,
    zeldovich_ics,
    zeldovich_displacement,
    lognormal_density,
    lognormal_particles,
    tophat_density,
    config_params,
    scan_params,
    pk_powerlaw_break,
    pk_sigma8_norm,
)
