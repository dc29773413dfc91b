"""GPU power spectrum (FFT, shell binning, CIC estimator grid) against the
oracle's NumPy estimator, and a single Fourier mode at every transform size,
where the answer is known in closed form."""
import numpy as np
import pytest

import oracle
from workloads import lattice_displacement_ics, lognormal_density

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2604_15434_amd as P

    return P


@pytest.mark.parametrize("n,dtype", [(8, torch.float64), (32, torch.float64), (64, torch.float32),
                                     (128, torch.float64), (256, torch.float64)])
def test_field_power_matches_oracle(P, n, dtype):
    """A lognormal field (rough at every scale): every shell up to n/2 within
    1e-11 relative (FP32 input: the same values widened) and the mode counts
    exact."""
    f = lognormal_density(n, 500.0 * n / 256, seed=7)
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    box = 300.0
    k_r, p_r, c_r = oracle.power_spectrum(f, box)
    k, p, c = P.pm_field_power(torch.from_numpy(f).to("cuda", dtype), box, nbins=n // 2)
    assert np.array_equal(c, c_r)
    np.testing.assert_allclose(k, k_r, rtol=1e-12)
    np.testing.assert_allclose(p, p_r, rtol=1e-11, atol=1e-13 * p_r.max())


@pytest.mark.parametrize("n", [16, 128, 512, 1024])
def test_single_mode_power(P, n):
    """f = cos(2 pi m.x) with m = (3, -1, 2) (|m| = sqrt 14, shell 3): only
    that shell has power, box^3 / 4 per mode of +-m, shared by the shell's
    count of modes; every other shell is zero to rounding.  Covers the
    transform at sizes the oracle comparison does not reach."""
    box = 100.0
    x = (torch.arange(n, dtype=torch.float64, device="cuda") / n).view(-1, 1, 1)
    y = (torch.arange(n, dtype=torch.float64, device="cuda") / n).view(1, -1, 1)
    z = (torch.arange(n, dtype=torch.float64, device="cuda") / n).view(1, 1, -1)
    f = torch.cos(2 * np.pi * (3 * x - y + 2 * z)).contiguous()
    nb = min(8, n // 2)
    k, p, c = P.pm_field_power(f, box, nbins=nb)
    m = np.arange(-(n // 2), n // 2)  # the grid's wave numbers per axis
    m2 = (m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2).ravel()
    counts = np.array([np.sum((m2 >= (b + 0.5) ** 2) & (m2 < (b + 1.5) ** 2)) for b in range(nb)])
    assert np.array_equal(c, counts)
    expect = np.zeros(nb)
    expect[3] = 2 * box**3 / 4 / counts[3]
    np.testing.assert_allclose(p, expect, rtol=1e-12, atol=1e-12 * expect.max())
    del f


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_particle_power_on_finer_grid_matches_oracle(P, dtype):
    """32^3 particles (lattice + displacement) deposited on a 64^3 estimator
    grid, shells below half its Nyquist wavenumber (nbins = n/4): against
    the oracle's CIC deposit and estimator."""
    pos = lattice_displacement_ics(32, 100.0, seed=0, rms_cells=0.6)
    if dtype == torch.float32:
        pos = pos.astype(np.float32).astype(np.float64)
    k_r, p_r, c_r = oracle.power_spectrum(oracle.density_contrast(oracle.cic_deposit(pos, 64)), 100.0)
    k, p, c = P.pm_particle_power(torch.from_numpy(pos).to("cuda", dtype), 64, 100.0)
    assert len(p) == 16 and np.array_equal(c, c_r[:16])
    np.testing.assert_allclose(p, p_r[:16], rtol=1e-9)


def test_boost_of_identical_runs_is_one(P):
    pos = torch.from_numpy(lattice_displacement_ics(32, 100.0, seed=1, rms_cells=0.4)).cuda()
    k, p, _ = P.pm_particle_power(pos, 64, 100.0)
    np.testing.assert_allclose(P.pm_boost(k, p, p, 0.028), 1.0, rtol=1e-15)
