"""The seeded input generators: the expected-variance normalisation of the
lognormal fields matches sample variances, and reference-grid normalisation
gives a smaller box the reference box's per-mode amplitude."""
import numpy as np
import pytest

from workloads import expected_variance, gaussian_field, lognormal_density
from workloads.ics import pk_powerlaw_break


def test_expected_variance_matches_samples():
    ng, box = 32, 62.5
    var = expected_variance(ng, box, pk_powerlaw_break)
    samples = [gaussian_field(ng, box, pk_powerlaw_break, seed=s).var() for s in range(40)]
    assert np.mean(samples) == pytest.approx(var, rel=0.03)


def test_reference_grid_normalisation():
    # a 256^3 / 500 Mpc/h box has std 1.5; a 64^3 box of the same cell size,
    # normalised to it, has the same per-mode amplitude and a smaller variance
    ref = (256, 500.0)
    s_ref = 1.5
    amp = s_ref / np.sqrt(expected_variance(*ref, pk_powerlaw_break))
    g = gaussian_field(64, 125.0, pk_powerlaw_break, seed=3) * amp
    expect = amp * np.sqrt(expected_variance(64, 125.0, pk_powerlaw_break))
    assert expect < s_ref
    rho = lognormal_density(64, 125.0, seed=3, ref_grid=ref)
    np.testing.assert_allclose(rho, np.exp(g - g.max()) / np.exp(g - g.max()).mean(), rtol=1e-12)
    assert rho.mean() == pytest.approx(1.0, rel=1e-12)
