"""Seeded synthetic initial conditions and parameter draws.

All fields are float64 NumPy arrays, C-order ``[i][j][k]`` with ``k``
fastest, on a periodic grid of ``ng`` cells per side whose cell ``(i,j,k)``
has its centre at ``((i+1/2)/ng, (j+1/2)/ng, (k+1/2)/ng)`` in box units.
Particle positions are returned as a ``(3, np)`` float64 array in ``[0, 1)``
box units (structure of arrays).

The paper's workloads use 2LPT initial conditions from CAMB spectra at
256^3-512^3 particles in a 328.125 Mpc/h box (Sec. 3.6, validation and
physical-study set-ups); those tools and data are not available, so the
analytic spectra below stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

OMEGA_M0 = 0.3071  # physical-study table (Sec. 3.6.3)


# ---------------------------------------------------------------- spectra
def pk_powerlaw_break(k, n=0.96, kb=0.05):
    """Unnormalised P(k) = k^n / (1 + (k/kb)^2)^2 (k in h/Mpc)."""
    k = np.asarray(k, dtype=np.float64)
    return k**n / (1.0 + (k / kb) ** 2) ** 2


def pk_sigma8_norm(shape=pk_powerlaw_break, radius=8.0, sigma=0.8):
    """Amplitude A such that A*shape(k) has a top-hat rms ``sigma`` at ``radius``.

    sigma^2(R) = 1/(2 pi^2) * int k^2 P(k) W^2(kR) dk with the spherical
    top-hat window W(x) = 3 (sin x - x cos x) / x^3, integrated on a fine
    logarithmic grid (trapezoid in ln k).
    """
    lnk = np.linspace(math.log(1e-5), math.log(1e2), 200001)
    k = np.exp(lnk)
    x = k * radius
    w = np.where(x < 1e-3, 1.0 - x**2 / 10.0, 3.0 * (np.sin(x) - x * np.cos(x)) / np.maximum(x, 1e-300) ** 3)
    integrand = k**3 * shape(k) * w**2 / (2.0 * math.pi**2)
    s2 = np.trapezoid(integrand, lnk)
    return sigma**2 / s2


# ---------------------------------------------------------------- grids
def _kvec(ng, box):
    """Wavevector components (h/Mpc) of an rfftn grid, broadcastable."""
    kf = 2.0 * math.pi / box
    k1 = np.fft.fftfreq(ng, d=1.0 / ng) * kf
    kr = np.fft.rfftfreq(ng, d=1.0 / ng) * kf
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kz = kr[None, None, :]
    return kx, ky, kz


def _nyquist_mask(ng):
    """Boolean rfftn-shaped mask that is False on the zero mode and Nyquist planes."""
    m1 = np.ones(ng, dtype=bool)
    mr = np.ones(ng // 2 + 1, dtype=bool)
    if ng % 2 == 0:
        m1[ng // 2] = False
        mr[ng // 2] = False
    mask = m1[:, None, None] & m1[None, :, None] & mr[None, None, :]
    mask[0, 0, 0] = False
    return mask


def _white_noise_hat(ng, rng):
    w = rng.standard_normal((ng, ng, ng))
    return np.fft.rfftn(w)


def gaussian_field(ng, box, pk, seed=None, rng=None):
    """Gaussian random field with power spectrum ``pk(k)`` (Mpc/h units).

    delta = irfftn(rfftn(w) * sqrt(P(k) ng^3 / L^3)) with w ~ N(0,1) per cell;
    the zero mode and the Nyquist planes are set to zero.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    wh = _white_noise_hat(ng, rng)
    kx, ky, kz = _kvec(ng, box)
    k = np.sqrt(kx**2 + ky**2 + kz**2)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = np.sqrt(pk(k[nz]) * ng**3 / box**3)
    dh = wh * amp * _nyquist_mask(ng)
    return np.fft.irfftn(dh, s=(ng, ng, ng), axes=(0, 1, 2))


def _lattice(ng):
    q1 = (np.arange(ng, dtype=np.float64) + 0.5) / ng
    qx, qy, qz = np.meshgrid(q1, q1, q1, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()])


# ---------------------------------------------------------------- particle loads
def lattice_displacement_ics(ng, box=100.0, seed=0, rms_cells=0.3, slope=-2.0):
    """Cell-centred lattice displaced by an irrotational Gaussian field.

    psi_hat = i k_hat sqrt(P(k)) w_hat with P(k) ~ k^slope, rescaled so the
    3-D rms displacement is ``rms_cells`` cells.  Returns (3, ng^3) positions.
    """
    rng = np.random.default_rng(seed)
    wh = _white_noise_hat(ng, rng)
    kx, ky, kz = _kvec(ng, box)
    k = np.sqrt(kx**2 + ky**2 + kz**2)
    mask = _nyquist_mask(ng)
    kk = np.where(k > 0, k, 1.0)
    amp = np.where(mask, kk ** (0.5 * slope), 0.0)
    psi = []
    for kc in (kx, ky, kz):
        ph = 1j * (kc / kk) * amp * wh
        psi.append(np.fft.irfftn(ph, s=(ng, ng, ng), axes=(0, 1, 2)).ravel())
    psi = np.stack(psi)
    rms = math.sqrt(np.mean(np.sum(psi**2, axis=0)))
    psi *= (rms_cells / ng) / rms
    return np.mod(_lattice(ng) + psi, 1.0)


def zeldovich_displacement(ng, box, seed, pk=None):
    """Lattice q (cell centres) and the Zel'dovich displacement field psi
    (psi_hat = i k delta_hat / k^2 of a Gaussian delta with spectrum ``pk``,
    default the sigma8 = 0.8 power-law-break one), both (3, ng^3) in box
    units; x = q + D psi moves the particles to growth factor D (D = 1 for
    the spectrum's normalisation)."""
    if pk is None:
        amp = pk_sigma8_norm()
        pk = lambda k: amp * pk_powerlaw_break(k)  # noqa: E731
    delta = gaussian_field(ng, box, pk, seed=seed)
    dh = np.fft.rfftn(delta)
    kx, ky, kz = _kvec(ng, box)
    k2 = kx**2 + ky**2 + kz**2
    k2[0, 0, 0] = 1.0
    psi = []
    for kc in (kx, ky, kz):
        ph = 1j * kc * dh / k2
        psi.append(np.fft.irfftn(ph, s=(ng, ng, ng), axes=(0, 1, 2)).ravel() / box)
    return _lattice(ng), np.stack(psi)


def zeldovich_ics(ng, box, seed, pk=None, np_side=None):
    """Zel'dovich particle load x = q + psi with psi_hat = i k delta_hat / k^2.

    ``pk`` defaults to the sigma8=0.8 normalised power-law-break spectrum.
    Positions of all (np_side^3) particles in box units, shape (3, np).
    """
    q, psi = zeldovich_displacement(ng if np_side is None else np_side, box, seed, pk)
    return np.mod(q + psi, 1.0)


def expected_variance(ng, box, pk):
    """Expected per-cell variance of gaussian_field(ng, box, pk): the sum of
    P(k) / L^3 over the modes it keeps (zero mode and Nyquist planes out)."""
    kx, ky, kz = _kvec(ng, box)
    k = np.sqrt(kx**2 + ky**2 + kz**2)
    p = np.zeros_like(k)
    nz = k > 0
    p[nz] = pk(k[nz])
    p = p * _nyquist_mask(ng)
    w = np.full(p.shape, 2.0)
    w[..., 0] = 1.0  # kz = 0 plane counted once; the Nyquist plane is masked
    return float(np.sum(w * p) / box**3)


def lognormal_density(ng, box, seed, sigma_g=1.5, pk=None, ref_grid=None):
    """Lognormal density rho = e^g / <e^g>.  g has std ``sigma_g`` in the box
    itself, or, with ref_grid = (ng_ref, box_ref), the amplitude that gives
    std sigma_g on that reference grid (same P(k) per mode: a smaller box of
    the same cell size then lacks only the long modes)."""
    if pk is None:
        pk = pk_powerlaw_break
    g = gaussian_field(ng, box, pk, seed=seed)
    if ref_grid is None:
        g *= sigma_g / g.std()
    else:
        g *= sigma_g / math.sqrt(expected_variance(ref_grid[0], ref_grid[1], pk))
    e = np.exp(g - g.max())
    return e / e.mean()


def lognormal_particles(ng, box, seed, sigma_g=1.5, n_particles=None):
    """Particles drawn multinomially from a lognormal density, uniform in cells.

    Returns (positions (3, np), rho_field).  Particles come out in cell order,
    which keeps neighbouring particles close in memory as a PM code's would be.
    """
    rng = np.random.default_rng(seed)
    g = gaussian_field(ng, box, pk_powerlaw_break, rng=rng)
    g *= sigma_g / g.std()
    e = np.exp(g - g.max())
    rho = e / e.mean()
    npart = ng**3 if n_particles is None else int(n_particles)
    cdf = np.cumsum(rho.ravel())
    cdf /= cdf[-1]
    cells = np.searchsorted(cdf, rng.random(npart), side="right")
    cells = np.minimum(cells, ng**3 - 1)
    cells.sort()
    i = cells // (ng * ng)
    j = (cells // ng) % ng
    kk = cells % ng
    off = rng.random((3, npart))
    pos = np.stack([(i + off[0]) / ng, (j + off[1]) / ng, (kk + off[2]) / ng])
    return np.mod(pos, 1.0), rho


def tophat_density(ng, radius_cells, delta_in, center=None):
    """Top-hat: rho = 1 + delta_in inside a sphere, compensated outside (mean 1).

    Cells are classified by their centre; ``center`` defaults to the box-centre
    vertex (ng/2, ng/2, ng/2) in cell units.
    """
    c = ng / 2.0 if center is None else center
    x = np.arange(ng) + 0.5 - c
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    inside = r2 < radius_cells**2
    n_in = inside.sum()
    rho = np.empty((ng, ng, ng))
    rho[inside] = 1.0 + delta_in
    rho[~inside] = 1.0 - delta_in * n_in / (ng**3 - n_in)
    return rho


# ---------------------------------------------------------------- parameters
def _p(ab, am, a, om=OMEGA_M0):
    return dict(omega_m0=om, alpha_b0=ab, alpha_m0=am, a=a)


def config_params(name):
    """Parameter sets of the named workload (list of dicts)."""
    if name == "cfg0":
        return [_p(-0.4, 0.0, 0.5)]
    if name == "cfg1":
        return [_p(ab, am, a) for ab in (-0.2, -0.6) for am in (0.0, 0.1) for a in (0.33, 1.0)]
    if name == "cfg2":
        return [_p(-0.2, 0.0, 1.0), _p(-0.6, 0.0, 1.0)]
    raise KeyError(name)


def scan_params(n, seed, a=None):
    """``n`` draws of alpha_B0 ~ U[-1,0], alpha_M0 ~ U[0,0.2] and a ~ U[0.2,1]
    (or fixed ``a``)."""
    rng = np.random.default_rng(seed)
    ab = rng.uniform(-1.0, 0.0, n)
    am = rng.uniform(0.0, 0.2, n)
    aa = rng.uniform(0.2, 1.0, n) if a is None else np.full(n, float(a))
    return [_p(float(x), float(y), float(z)) for x, y, z in zip(ab, am, aa)]
