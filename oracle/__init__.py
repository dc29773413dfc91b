"""CPU oracle of the EFTofDE particle-mesh gravity step (float64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls this package; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the HIP path: the two meet only at the
seeded inputs of ``workloads``.

* ``coeffs``  -- background/EFT coefficients (Secs. 2.2-2.6, 3.1), growth
  ODE (eq. delta_mod_a), static spherical closed form (eq. analytical).
* ``fields``  -- CIC deposit/interpolation, exact FFT Poisson solve of the
  7-point Laplacian, 5-point gradient, power spectrum.
* ``solver``  -- the nonlinear scalar-field FAS multigrid (plain C, see
  ``csrc/chi_fas.c``) and the full PM step.

Parity pins (what fixes each function independently of itself) live in
``tests/test_oracle_*.py``.
"""
from .coeffs import eft_coefficients, growth_factor, spherical_x, spherical_yz  # noqa: F401
from .fields import (  # noqa: F401
    cic_deposit,
    cic_interpolate,
    density_contrast,
    gradient5,
    laplacian7,
    poisson_fft,
    power_spectrum,
)
from .solver import (  # noqa: F401
    chi_operator,
    fas_solve,
    pm_step,
    relative_residual,
    solve_chi,
    solve_chi_linear,
    solve_poisson,
)
